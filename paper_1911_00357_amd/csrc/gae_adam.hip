// GAE reverse scan, advantage statistics (float64) and the fused Adam step.
#include "common.h"
#include "kernels.h"

// ---------------------------------------------------------------------------
// GAE (Sec. 4 "Training"; Schulman et al. 2015).  One wavefront per env.  The
// recurrence A_t = delta_t + c_t A_{t+1} (c_t = gamma lambda (1 - d_t)) is a
// composition of affine maps, so each 64-step chunk is solved with a suffix
// scan across lanes (lane = time step), chunks walked from the end; steps at
// or past len[n] have delta = c = 0, which leaves A = 0 there.
__global__ void __launch_bounds__(256) gae_kernel(const float* __restrict__ rew,
                                                  const float* __restrict__ val,
                                                  const uint8_t* __restrict__ done,
                                                  const int32_t* __restrict__ len, int T, int N,
                                                  float gamma, float lambda, float* __restrict__ adv,
                                                  float* __restrict__ ret) {
  const int lane = threadIdx.x & 63;
  const int n = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (n >= N) return;
  const int Tn = len ? min(max(len[n], 0), T) : T;
  float carry = 0.f;  // A at the first step of the chunk after this one
  const int nchunks = (T + 63) / 64;
  for (int ch = nchunks - 1; ch >= 0; --ch) {
    const int t = ch * 64 + lane;
    float a = 0.f, b = 0.f, v = 0.f;
    if (t < Tn) {
      const float keep = done[(size_t)t * N + n] ? 0.f : 1.f;
      v = val[(size_t)t * N + n];
      b = rew[(size_t)t * N + n] + gamma * keep * val[(size_t)(t + 1) * N + n] - v;
      a = gamma * lambda * keep;
    }
    // inclusive suffix scan of f_t o f_{t+1} o ... : (a, b) with F(x) = b + a x
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const float a2 = __shfl_down(a, o, 64);
      const float b2 = __shfl_down(b, o, 64);
      if (lane + o < 64) {
        b = b + a * b2;
        a = a * a2;
      }
    }
    const float A = b + a * carry;
    if (t < T) {
      adv[(size_t)t * N + n] = A;
      ret[(size_t)t * N + n] = (t < Tn) ? A + v : 0.f;
    }
    carry = __shfl(A, 0, 64);
  }
}

// Population mean / variance of the valid advantages in float64 (two passes),
// one workgroup.
__global__ void __launch_bounds__(256) adv_stats_kernel(const float* __restrict__ adv,
                                                        const int32_t* __restrict__ len, int T,
                                                        int N, double* __restrict__ out) {
  __shared__ double red[4];
  __shared__ double s_mean;
  const int tid = threadIdx.x;
  double s = 0.0, cnt = 0.0;
  for (int i = tid; i < T * N; i += 256) {
    const int t = i / N, n = i % N;
    const int Tn = len ? len[n] : T;
    if (t < Tn) {
      s += (double)adv[i];
      cnt += 1.0;
    }
  }
  s = wave_sum(s);
  cnt = wave_sum(cnt);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  double total = red[0] + red[1] + red[2] + red[3];
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = cnt;
  __syncthreads();
  const double count = red[0] + red[1] + red[2] + red[3];
  if (tid == 0) s_mean = count > 0 ? total / count : 0.0;
  __syncthreads();
  const double mean = s_mean;
  double q = 0.0;
  for (int i = tid; i < T * N; i += 256) {
    const int t = i / N, n = i % N;
    const int Tn = len ? len[n] : T;
    if (t < Tn) {
      const double d = (double)adv[i] - mean;
      q += d * d;
    }
  }
  q = wave_sum(q);
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = q;
  __syncthreads();
  if (tid == 0) {
    out[0] = mean;
    out[1] = count > 0 ? (red[0] + red[1] + red[2] + red[3]) / count : 0.0;
  }
}

void launch_gae(const float* rew, const float* val, const uint8_t* done, const int32_t* len,
                int T, int N, float gamma, float lambda, float* adv, float* ret, double* stats,
                hipStream_t s) {
  hipLaunchKernelGGL(gae_kernel, dim3(cdiv(N, 4)), dim3(256), 0, s, rew, val, done, len, T, N,
                     gamma, lambda, adv, ret);
  if (stats) hipLaunchKernelGGL(adv_stats_kernel, dim3(1), dim3(256), 0, s, adv, len, T, N, stats);
}

// ---------------------------------------------------------------------------
// Adam with dynamic loss scaling.  Three launches, no host synchronisation:
//   1. per-block "any non-finite gradient" flags
//   2. one workgroup folds the flags, updates the scaler and writes the step
//      constants (1/S, bias corrections, skip) to the workspace
//   3. the elementwise update (and the bfloat16 re-cast of the master).
struct AdamConsts {
  float inv_scale;
  float c1;  // 1 / (1 - b1^k)
  float c2;  // 1 / (1 - b2^k)
  int skip;
};

constexpr int kAdamBlocks = 1024;

__global__ void __launch_bounds__(256) adam_check_kernel(const float* __restrict__ g, size_t P,
                                                         const ppo_scaler* sc,
                                                         int* __restrict__ flags) {
  const float inv = 1.0f / sc->scale;
  int bad = 0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < P; i += (size_t)gridDim.x * 256) {
    const float x = g[i] * inv;
    bad |= !isfinite(x);
  }
  bad = __syncthreads_or(bad);
  if (threadIdx.x == 0) flags[blockIdx.x] = bad;
}

__global__ void __launch_bounds__(256) adam_finalize_kernel(const int* __restrict__ flags, int nflags,
                                                            ppo_scaler* sc, float b1, float b2,
                                                            int growth, AdamConsts* out) {
  int bad = 0;
  for (int i = threadIdx.x; i < nflags; i += 256) bad |= flags[i];
  bad = __syncthreads_or(bad);
  if (threadIdx.x == 0) {
    AdamConsts c;
    c.inv_scale = 1.0f / sc->scale;
    c.skip = bad;
    if (bad) {
      if (growth > 0) sc->scale = sc->scale * 0.5f;  // a static scale (growth 0) stays fixed
      sc->good_steps = 0;
      sc->skipped += 1;
      sc->found_inf = 1;
      c.c1 = c.c2 = 0.f;
    } else {
      const int k = sc->step + 1;
      sc->step = k;
      sc->found_inf = 0;
      // 1 / (1 - b^k) = -1 / expm1(k log1p(b - 1)); b - 1 is exact in float for b in [0.5, 1)
      c.c1 = -1.0f / expm1f((float)k * log1pf(b1 - 1.0f));
      c.c2 = -1.0f / expm1f((float)k * log1pf(b2 - 1.0f));
      if (growth > 0) {
        sc->good_steps += 1;
        if (sc->good_steps >= growth) {
          sc->scale = sc->scale * 2.0f;
          sc->good_steps = 0;
        }
      }
    }
    *out = c;
  }
}

__global__ void __launch_bounds__(256) adam_update_kernel(float* __restrict__ th,
                                                          const float* __restrict__ g,
                                                          float* __restrict__ m, float* __restrict__ v,
                                                          bf16_t* __restrict__ lp, size_t P, float lr,
                                                          float b1, float b2, float eps,
                                                          const AdamConsts* cst) {
  const AdamConsts c = *cst;
  if (c.skip) return;
  const size_t stride = (size_t)gridDim.x * 256 * 4;
  for (size_t i0 = ((size_t)blockIdx.x * 256 + threadIdx.x) * 4; i0 < P; i0 += stride) {
    if (i0 + 4 <= P) {
      float4 gg = *(const float4*)(g + i0);
      float4 mm = *(const float4*)(m + i0);
      float4 vv = *(const float4*)(v + i0);
      float4 tt = *(const float4*)(th + i0);
      float gs[4] = {gg.x, gg.y, gg.z, gg.w}, ms[4] = {mm.x, mm.y, mm.z, mm.w},
            vs[4] = {vv.x, vv.y, vv.z, vv.w}, ts[4] = {tt.x, tt.y, tt.z, tt.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float gj = gs[j] * c.inv_scale;
        ms[j] = b1 * ms[j] + (1.f - b1) * gj;
        vs[j] = b2 * vs[j] + (1.f - b2) * gj * gj;
        ts[j] -= lr * (ms[j] * c.c1) / (sqrtf(vs[j] * c.c2) + eps);
      }
      *(float4*)(m + i0) = make_float4(ms[0], ms[1], ms[2], ms[3]);
      *(float4*)(v + i0) = make_float4(vs[0], vs[1], vs[2], vs[3]);
      *(float4*)(th + i0) = make_float4(ts[0], ts[1], ts[2], ts[3]);
      if (lp) {
#pragma unroll
        for (int j = 0; j < 4; ++j) lp[i0 + j] = f2bf(ts[j]);
      }
    } else {
      for (size_t i = i0; i < P; ++i) {
        const float gj = g[i] * c.inv_scale;
        m[i] = b1 * m[i] + (1.f - b1) * gj;
        v[i] = b2 * v[i] + (1.f - b2) * gj * gj;
        th[i] -= lr * (m[i] * c.c1) / (sqrtf(v[i] * c.c2) + eps);
        if (lp) lp[i] = f2bf(th[i]);
      }
    }
  }
}

__global__ void __launch_bounds__(256) cast_bf16_kernel(const float* __restrict__ src,
                                                        bf16_t* __restrict__ dst, size_t n) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    dst[i] = f2bf(src[i]);
}

size_t adam_ws_bytes() { return 256 + kAdamBlocks * sizeof(int); }

void launch_adam(float* th, const float* g, float* m, float* v, bf16_t* lp, size_t P, float lr,
                 float b1, float b2, float eps, int growth, ppo_scaler* sc, void* ws,
                 hipStream_t s) {
  AdamConsts* cst = (AdamConsts*)ws;
  int* flags = (int*)((char*)ws + 256);
  const int nb = (int)std::min<size_t>(kAdamBlocks, (P + 255) / 256);
  hipLaunchKernelGGL(adam_check_kernel, dim3(nb), dim3(256), 0, s, g, P, sc, flags);
  hipLaunchKernelGGL(adam_finalize_kernel, dim3(1), dim3(256), 0, s, flags, nb, sc, b1, b2, growth,
                     cst);
  const int nu = (int)std::min<size_t>(4096, (P + 1023) / 1024);
  hipLaunchKernelGGL(adam_update_kernel, dim3(nu), dim3(256), 0, s, th, g, m, v, lp, P, lr, b1, b2,
                     eps, cst);
}

void launch_cast_bf16(const float* src, bf16_t* dst, size_t n, hipStream_t s) {
  const int nb = (int)std::min<size_t>(4096, (n + 255) / 256);
  hipLaunchKernelGGL(cast_bf16_kernel, dim3(nb), dim3(256), 0, s, src, dst, n);
}
