// GAE reverse scan, advantage statistics (float64) and the fused Adam step.
#include "common.h"
#include "kernels.h"

// ---------------------------------------------------------------------------
// GAE (Sec. 4 "Training"; Schulman et al. 2015).  A workgroup covers 64 envs.
// The rollout is walked in 64-step chunks from the end; each chunk of rew,
// done and val ([T][N] rows, val one row longer) is staged through LDS with
// loads coalesced along the env axis, and the results leave the same way.
// Each wavefront then solves the recurrence A_t = delta_t + c_t A_{t+1}
// (c_t = gamma lambda (1 - d_t)) for 16 of the envs, one at a time: it is a
// composition of affine maps, so a chunk is a suffix scan across lanes
// (lane = time step) continued from the carried A of the chunk after it;
// steps at or past len[n] have delta = c = 0, which leaves A = 0 there.
constexpr int kGaeEnvs = 64;
__global__ void __launch_bounds__(256) gae_kernel(const float* __restrict__ rew,
                                                  const float* __restrict__ val,
                                                  const uint8_t* __restrict__ done,
                                                  const int32_t* __restrict__ len, int T, int N,
                                                  float gamma, float lambda, float* __restrict__ adv,
                                                  float* __restrict__ ret) {
  // [t][env], rows padded to 65 so that a wavefront reading one env's column
  // (lane = t) touches 64 different banks; s_r / s_k are overwritten in place
  // by A and the return
  __shared__ float s_r[64][kGaeEnvs + 1], s_k[64][kGaeEnvs + 1], s_v[65][kGaeEnvs + 1];
  __shared__ float s_carry[kGaeEnvs];
  __shared__ int s_len[kGaeEnvs];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int n0 = blockIdx.x * kGaeEnvs;
  if (tid < kGaeEnvs) {
    const int n = n0 + tid;
    s_carry[tid] = 0.f;  // A at the first step of the chunk after this one
    s_len[tid] = n < N ? (len ? min(max(len[n], 0), T) : T) : 0;
  }
  const int nchunks = (T + 63) / 64;
  for (int ch = nchunks - 1; ch >= 0; --ch) {
    const int t0 = ch * 64;
    __syncthreads();  // the previous chunk's results have left s_r / s_k
    for (int i = tid; i < 65 * kGaeEnvs; i += 256) {
      const int r = i / kGaeEnvs, c = i - r * kGaeEnvs, t = t0 + r, n = n0 + c;
      const bool in = n < N;
      if (r < 64) {
        s_r[r][c] = in && t < T ? rew[(size_t)t * N + n] : 0.f;
        s_k[r][c] = in && t < T ? (done[(size_t)t * N + n] ? 0.f : 1.f) : 0.f;
      }
      s_v[r][c] = in && t <= T ? val[(size_t)t * N + n] : 0.f;
    }
    __syncthreads();
    for (int j = w; j < kGaeEnvs && n0 + j < N; j += 4) {
      const int t = t0 + lane, Tn = s_len[j];
      float a = 0.f, b = 0.f, v = 0.f;
      if (t < Tn) {
        const float keep = s_k[lane][j];
        v = s_v[lane][j];
        b = s_r[lane][j] + gamma * keep * s_v[lane + 1][j] - v;
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
      const float A = b + a * s_carry[j];
      s_r[lane][j] = A;
      s_k[lane][j] = t < Tn ? A + v : 0.f;
      const float first = __shfl(A, 0, 64);
      if (lane == 0) s_carry[j] = first;
    }
    __syncthreads();
    for (int i = tid; i < 64 * kGaeEnvs; i += 256) {
      const int r = i / kGaeEnvs, c = i - r * kGaeEnvs, t = t0 + r, n = n0 + c;
      if (t < T && n < N) {
        adv[(size_t)t * N + n] = s_r[r][c];
        ret[(size_t)t * N + n] = s_k[r][c];
      }
    }
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
  hipLaunchKernelGGL(gae_kernel, dim3(cdiv(N, kGaeEnvs)), dim3(256), 0, s, rew, val, done, len, T, N,
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
