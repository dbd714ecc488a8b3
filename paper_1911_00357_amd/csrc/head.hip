// Policy/value head, action sampling, the PPO loss with its gradient, the
// goal / previous-action inputs of the LSTM, and minibatch bookkeeping.
#include "common.h"
#include "kernels.h"

constexpr int kMaxA = 8;  // actions + value row handled per wavefront

// Goal feature k of one frame (goal modes: 0 raw 2-vector, 1 polar
// (d, theta) -> [d, cos, sin] -> FC, 2 a given 3-vector -> FC; 3 none).
DEV float goal_feature(const float* __restrict__ goal, size_t si, int gmode, int k, const float* __restrict__ gw,
                       const float* __restrict__ gb) {
  if (gmode == 2) {
    const float* g3 = goal + si * 3;
    return gb[k] + gw[k * 3] * g3[0] + gw[k * 3 + 1] * g3[1] + gw[k * 3 + 2] * g3[2];
  }
  const float d = goal[si * 2], th = goal[si * 2 + 1];
  if (gmode == 1) return gb[k] + gw[k * 3] * d + gw[k * 3 + 1] * cosf(th) + gw[k * 3 + 2] * sinf(th);
  return (k == 0) ? d : th;
}

// Input i of the goal FC for one frame (polar or 3-vector mode).
DEV float goal_input(const float* __restrict__ goal, size_t si, int gmode, int i) {
  if (gmode == 2) return goal[si * 3 + i];
  const float d = goal[si * 2], th = goal[si * 2 + 1];
  return (i == 0) ? d : (i == 1 ? cosf(th) : sinf(th));
}

// One wavefront per row: out[k] = W[k] . h + b[k] for k < A+1.
DEV void head_dots(const float* __restrict__ h, const float* __restrict__ W, const float* __restrict__ b,
                   int H, int A1, float out[kMaxA]) {
  const int lane = threadIdx.x & 63;
  float acc[kMaxA];
#pragma unroll
  for (int k = 0; k < kMaxA; ++k) acc[k] = 0.f;
  // branch-free loads (rows k >= A1 re-read row A1-1 and are discarded), so
  // the loads of an iteration, and of the unrolled iterations, are in flight together
#pragma unroll 4
  for (int j = lane; j < H; j += 64) {
    const float hv = h[j];
#pragma unroll
    for (int k = 0; k < kMaxA; ++k) acc[k] += W[(size_t)min(k, A1 - 1) * H + j] * hv;
  }
#pragma unroll
  for (int k = 0; k < kMaxA; ++k) out[k] = (k < A1) ? wave_sum(acc[k]) + b[k] : 0.f;
}

// One wavefront per row: dh[j] = sum_{k < A1} d[k] W[k][j] (d[k] = 0 for k >= A1).
DEV void head_dh(const float d[kMaxA], const float* __restrict__ W, int H, int A1, float* __restrict__ dh) {
  const int lane = threadIdx.x & 63;
#pragma unroll 4
  for (int j = lane; j < H; j += 64) {
    float v = 0.f;
#pragma unroll
    for (int k = 0; k < kMaxA; ++k) v += d[k] * W[(size_t)min(k, A1 - 1) * H + j];
    dh[j] = v;
  }
}

// Act head: logits, value, log-softmax, inverse-CDF sample.
__global__ void __launch_bounds__(256) act_head_kernel(const float* __restrict__ htop, int rows, int H,
                                                       int A, const float* __restrict__ W,
                                                       const float* __restrict__ bias,
                                                       const float* __restrict__ u,
                                                       int32_t* __restrict__ action,
                                                       float* __restrict__ logp, float* __restrict__ value,
                                                       float* __restrict__ logits,
                                                       const int32_t* __restrict__ active) {
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  // rows >= *active (a device count, read when the kernel runs) are not written
  if (r >= rows || (active && r >= *active)) return;
  float o[kMaxA];
  head_dots(htop + (size_t)r * H, W, bias, H, A + 1, o);
  if (lane == 0) {
    float mx = o[0];
    for (int k = 1; k < A; ++k) mx = fmaxf(mx, o[k]);
    float se = 0.f;
    for (int k = 0; k < A; ++k) se += expf(o[k] - mx);
    const float lse = mx + logf(se);
    const float uu = u[r];
    int a = A - 1;
    float cdf = 0.f;
    for (int k = 0; k < A; ++k) {
      cdf += expf(o[k] - lse);
      if (cdf > uu) {
        a = k;
        break;
      }
    }
    action[r] = a;
    logp[r] = o[a] - lse;
    value[r] = o[A];
    if (logits)
      for (int k = 0; k < A; ++k) logits[(size_t)r * A + k] = o[k];
  }
}

void launch_act_head(const float* htop, int rows, int H, int A, const float* W, const float* b,
                     const float* u, int32_t* action, float* logp, float* value, float* logits,
                     const int32_t* active, hipStream_t s) {
  hipLaunchKernelGGL(act_head_kernel, dim3(cdiv(rows, 4)), dim3(256), 0, s, htop, rows, H, A, W, b, u,
                     action, logp, value, logits, active);
}

// PPO loss terms of one frame (Eq. 2 with ratio r = exp(logp - logp_old);
// value term 1/2 (V - R)^2; entropy bonus) with frame weight w, from its
// logits o[0..A) and value o[A]:
//   fs[0..6) = {w(-min(rA, clip(r)A)), w 1/2 (V-R)^2, w H, w [|r-1| > eps], w (lp_old - lp), r}
//   d[0..A]  = S * dL/d(logits, value)
DEV void ppo_frame_terms(const float o[kMaxA], int A, int a, float At, float lp_old, float R, float w,
                         float clip, float vcoef, float ecoef, float S, float d[kMaxA], float fs[6]) {
  float mx = o[0];
  for (int k = 1; k < A; ++k) mx = fmaxf(mx, o[k]);
  float se = 0.f;
  for (int k = 0; k < A; ++k) se += expf(o[k] - mx);
  const float lse = mx + logf(se);
  const float lpa = o[a] - lse;
  const float ratio = expf(lpa - lp_old);
  const float s1 = ratio * At;
  const float s2 = fminf(fmaxf(ratio, 1.f - clip), 1.f + clip) * At;
  const float surr = fminf(s1, s2);
  float ent = 0.f;
  float p[kMaxA], lp[kMaxA];
  for (int k = 0; k < A; ++k) {
    lp[k] = o[k] - lse;
    p[k] = expf(lp[k]);
    ent -= p[k] * lp[k];
  }
  const float V = o[A];
  // d/dlogp(a): the unclipped branch (taken at ties) carries r A
  const float dlpa = (s1 <= s2) ? -w * At * ratio : 0.f;
#pragma unroll
  for (int k = 0; k < kMaxA; ++k) d[k] = 0.f;
  for (int k = 0; k < A; ++k) {
    const float onehot = (k == a) ? 1.f : 0.f;
    d[k] = S * (dlpa * (onehot - p[k]) + ecoef * w * p[k] * (lp[k] + ent));
  }
  d[A] = S * vcoef * w * (V - R);
  fs[0] = -w * surr;
  fs[1] = w * 0.5f * (V - R) * (V - R);
  fs[2] = w * ent;
  fs[3] = (fabsf(ratio - 1.f) > clip) ? w : 0.f;
  fs[4] = w * (lp_old - lpa);
  fs[5] = ratio;
}

// the advantage of a frame, normalised with the float64 statistics of ppo_gae
// (read once, then float32 arithmetic) when norm_adv is set
DEV float frame_adv(const float* adv, int sidx, int norm_adv, const double* adv_stats) {
  const float At = adv[sidx];
  if (!norm_adv) return At;
  const float mean = (float)adv_stats[0], sd = sqrtf((float)adv_stats[1]);
  return (At - mean) / (sd + 1e-5f);
}

// Learner head + PPO loss, one wavefront per frame f:
//   fstat[f] = ppo_frame_terms' fs; dout[f] = its d; dh[f] = dout[f] W (gradient
//   into the top LSTM output)
__global__ void __launch_bounds__(256) loss_head_kernel(
    const float* __restrict__ htop, int F, int H, int A, const float* __restrict__ W,
    const float* __restrict__ bias, const int32_t* __restrict__ src, const int32_t* __restrict__ actions,
    const float* __restrict__ logp_old, const float* __restrict__ adv, const float* __restrict__ ret,
    const float* __restrict__ wf, float clip, float vcoef, float ecoef, int norm_adv,
    const double* __restrict__ adv_stats, const float* __restrict__ loss_scale,
    float* __restrict__ fstat, float* __restrict__ dout, float* __restrict__ dh) {
  const int f = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (f >= F) return;
  float o[kMaxA];
  head_dots(htop + (size_t)f * H, W, bias, H, A + 1, o);
  const int sidx = src[f];
  float d[kMaxA], fs[6];
  // every lane computes the (scalar) loss terms; lane 0 stores them
  ppo_frame_terms(o, A, actions[sidx], frame_adv(adv, sidx, norm_adv, adv_stats), logp_old[sidx], ret[sidx],
                  wf[f], clip, vcoef, ecoef, loss_scale ? *loss_scale : 1.f, d, fs);
  if (lane == 0) {
    for (int k = 0; k < 6; ++k) fstat[(size_t)f * 8 + k] = fs[k];
    for (int k = 0; k <= A; ++k) dout[(size_t)f * (A + 1) + k] = d[k];
  }
  head_dh(d, W, H, A + 1, dh + (size_t)f * H);
}

// PPO loss on given policy outputs, one thread per frame: logits [F][A],
// values [F] in, fstat as above, dlogits [F][A] and dvalues [F] out.
__global__ void __launch_bounds__(256) loss_terms_kernel(
    const float* __restrict__ logits, const float* __restrict__ values, int F, int A,
    const int32_t* __restrict__ src, const int32_t* __restrict__ actions, const float* __restrict__ logp_old,
    const float* __restrict__ adv, const float* __restrict__ ret, const float* __restrict__ wf, float clip,
    float vcoef, float ecoef, int norm_adv, const double* __restrict__ adv_stats,
    const float* __restrict__ loss_scale, float* __restrict__ fstat, float* __restrict__ dlogits,
    float* __restrict__ dvalues) {
  const int f = blockIdx.x * 256 + threadIdx.x;
  if (f >= F) return;
  float o[kMaxA];
#pragma unroll
  for (int k = 0; k < kMaxA; ++k) o[k] = 0.f;
  for (int k = 0; k < A; ++k) o[k] = logits[(size_t)f * A + k];
  o[A] = values[f];
  const int sidx = src[f];
  float d[kMaxA], fs[6];
  ppo_frame_terms(o, A, actions[sidx], frame_adv(adv, sidx, norm_adv, adv_stats), logp_old[sidx], ret[sidx],
                  wf[f], clip, vcoef, ecoef, loss_scale ? *loss_scale : 1.f, d, fs);
  for (int k = 0; k < 6; ++k) fstat[(size_t)f * 8 + k] = fs[k];
  for (int k = 0; k < A; ++k) dlogits[(size_t)f * A + k] = d[k];
  dvalues[f] = d[A];
}

// stats[8] = {loss, pg, vf, ent, clip_frac, approx_kl, ratio_min, ratio_max}
// loss_out (or NULL): S * stats[0], S = *loss_scale (1 when NULL).
__global__ void __launch_bounds__(256) loss_stats_kernel(const float* __restrict__ fstat, int F,
                                                         float vcoef, float ecoef,
                                                         float* __restrict__ stats,
                                                         const float* __restrict__ loss_scale,
                                                         float* __restrict__ loss_out) {
  __shared__ float red[5][4];
  __shared__ float rmn[4], rmx[4];
  float acc[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
  float mn = INFINITY, mx = -INFINITY;
  for (int f = threadIdx.x; f < F; f += 256) {
    const float* fs = fstat + (size_t)f * 8;
    for (int k = 0; k < 5; ++k) acc[k] += fs[k];
    mn = fminf(mn, fs[5]);
    mx = fmaxf(mx, fs[5]);
  }
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int k = 0; k < 5; ++k) acc[k] = wave_sum(acc[k]);
  for (int o = 32; o > 0; o >>= 1) {
    mn = fminf(mn, __shfl_xor(mn, o, 64));
    mx = fmaxf(mx, __shfl_xor(mx, o, 64));
  }
  if (lane == 0) {
    for (int k = 0; k < 5; ++k) red[k][w] = acc[k];
    rmn[w] = mn;
    rmx[w] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float t[5];
    for (int k = 0; k < 5; ++k) t[k] = (red[k][0] + red[k][1]) + (red[k][2] + red[k][3]);
    const float loss = t[0] + vcoef * t[1] - ecoef * t[2];
    stats[0] = loss;
    for (int k = 0; k < 5; ++k) stats[1 + k] = t[k];
    if (loss_out) *loss_out = loss * (loss_scale ? *loss_scale : 1.f);
    stats[6] = fminf(fminf(rmn[0], rmn[1]), fminf(rmn[2], rmn[3]));
    stats[7] = fmaxf(fmaxf(rmx[0], rmx[1]), fmaxf(rmx[2], rmx[3]));
  }
}

void launch_loss_head(const float* htop, int F, int H, int A, const float* W, const float* b,
                      const int32_t* src, const int32_t* actions, const float* logp_old,
                      const float* adv, const float* ret, const float* wf, float clip, float vcoef,
                      float ecoef, int norm_adv, const double* adv_stats, const float* loss_scale,
                      float* fstat, float* dout, float* dh, float* stats, hipStream_t s) {
  hipLaunchKernelGGL(loss_head_kernel, dim3(cdiv(F, 4)), dim3(256), 0, s, htop, F, H, A, W, b, src,
                     actions, logp_old, adv, ret, wf, clip, vcoef, ecoef, norm_adv, adv_stats, loss_scale,
                     fstat, dout, dh);
  hipLaunchKernelGGL(loss_stats_kernel, dim3(1), dim3(256), 0, s, fstat, F, vcoef, ecoef, stats, nullptr,
                     nullptr);
}

void launch_loss_terms(const float* logits, const float* values, int F, int A, const int32_t* src,
                       const int32_t* actions, const float* logp_old, const float* adv, const float* ret,
                       const float* wf, float clip, float vcoef, float ecoef, int norm_adv,
                       const double* adv_stats, const float* loss_scale, float* fstat, float* dlogits,
                       float* dvalues, float* stats, float* loss_out, hipStream_t s) {
  hipLaunchKernelGGL(loss_terms_kernel, dim3(cdiv(F, 256)), dim3(256), 0, s, logits, values, F, A, src, actions,
                     logp_old, adv, ret, wf, clip, vcoef, ecoef, norm_adv, adv_stats, loss_scale, fstat, dlogits,
                     dvalues);
  hipLaunchKernelGGL(loss_stats_kernel, dim3(1), dim3(256), 0, s, fstat, F, vcoef, ecoef, stats, loss_scale,
                     loss_out);
}

// --------------------------------------------------------- LSTM input parts
// Z[f][zoff + k]: goal features (polar: FC over [d, cos, sin]; raw: the
// 2-vector) and the previous-action embedding (row 0 = start token when the
// episode mask is 0).  Inputs of frame f are read at index src[f] (or f).
__global__ void __launch_bounds__(256) embed_fwd_kernel(const float* __restrict__ goal,
                                                        const int32_t* __restrict__ prev_a,
                                                        const float* __restrict__ mask,
                                                        const int32_t* __restrict__ src, int F, int polar,
                                                        int goal_dim, const float* __restrict__ gw,
                                                        const float* __restrict__ gb, int E,
                                                        const float* __restrict__ emb, float* __restrict__ Z,
                                                        int ldz, int zoff) {
  const int per = goal_dim + E;
  const int n = F * per;
  for (int e = blockIdx.x * 256 + threadIdx.x; e < n; e += gridDim.x * 256) {
    const int f = e / per, k = e - f * per;
    const int si = src ? src[f] : f;
    float v;
    if (k < goal_dim) {
      v = goal_feature(goal, (size_t)si, polar, k, gw, gb);
    } else {
      const int j = k - goal_dim;
      const int idx = (mask[si] == 0.f) ? 0 : prev_a[si] + 1;
      v = emb[(size_t)idx * E + j];
    }
    Z[(size_t)f * ldz + zoff + k] = v;
  }
}

void launch_embed_fwd(const float* goal, const int32_t* prev_a, const float* mask, const int32_t* src,
                      int F, int polar, int goal_dim, const float* gw, const float* gb, int E,
                      const float* emb, float* Z, int ldz, int zoff, hipStream_t s) {
  const int n = F * (goal_dim + E);
  if (n <= 0) return;
  hipLaunchKernelGGL(embed_fwd_kernel, dim3(std::min(4096, cdiv(n, 256))), dim3(256), 0, s, goal, prev_a,
                     mask, src, F, polar, goal_dim, gw, gb, E, emb, Z, ldz, zoff);
}

// Gradients of the goal FC (polar) and the embedding table: one wavefront per
// output element, frames summed in a fixed order.
__global__ void __launch_bounds__(256) embed_bwd_kernel(const float* __restrict__ goal,
                                                        const int32_t* __restrict__ prev_a,
                                                        const float* __restrict__ mask,
                                                        const int32_t* __restrict__ src, int F,
                                                        int polar, int goal_dim, int E, int A1,
                                                        const float* __restrict__ dZ, int ldz, int zoff,
                                                        float* __restrict__ dgw, float* __restrict__ dgb,
                                                        float* __restrict__ demb) {
  const int wid = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int ngoal = (polar == 1 || polar == 2) ? goal_dim * 4 : 0;
  const int nemb = A1 * E;
  if (wid >= ngoal + nemb) return;
  float acc = 0.f;
  if (wid < ngoal) {
    const int k = wid / 4, i = wid % 4;  // i < 3: weight column, i = 3: bias
    for (int f = lane; f < F; f += 64) {
      const int si = src ? src[f] : f;
      const float g = dZ[(size_t)f * ldz + zoff + k];
      const float x = i < 3 ? goal_input(goal, (size_t)si, polar, i) : 1.f;
      acc = fmaf(g, x, acc);
    }
    acc = wave_sum(acc);
    if (lane == 0) {
      if (i < 3) dgw[k * 3 + i] = acc;
      else dgb[k] = acc;
    }
  } else {
    const int q = wid - ngoal, a = q / E, j = q % E;
    for (int f = lane; f < F; f += 64) {
      const int si = src ? src[f] : f;
      const int idx = (mask[si] == 0.f) ? 0 : prev_a[si] + 1;
      if (idx == a) acc += dZ[(size_t)f * ldz + zoff + goal_dim + j];
    }
    acc = wave_sum(acc);
    if (lane == 0) demb[(size_t)a * E + j] = acc;
  }
}

void launch_embed_bwd(const float* goal, const int32_t* prev_a, const float* mask, const int32_t* src,
                      int F, int polar, int goal_dim, int E, int A1, const float* dZ, int ldz, int zoff,
                      float* dgw, float* dgb, float* demb, hipStream_t s) {
  const int n = ((polar == 1 || polar == 2) ? goal_dim * 4 : 0) + (E > 0 ? A1 * E : 0);
  if (n <= 0) return;
  hipLaunchKernelGGL(embed_bwd_kernel, dim3(cdiv(n, 4)), dim3(256), 0, s, goal, prev_a, mask, src, F,
                     polar, goal_dim, E > 0 ? E : 1, E > 0 ? A1 : 0, dZ, ldz, zoff, dgw, dgb, demb);
}

// dx[r][c] = dy[r][c] * [y[r][c] > 0] over a [rows][cols] window with row strides.
__global__ void __launch_bounds__(256) relu_grad2d_kernel(const float* __restrict__ dy, int ldd,
                                                          const float* __restrict__ y, int ldy, int rows,
                                                          int cols, float* __restrict__ dx, int ldx) {
  const int n = rows * cols;
  for (int e = blockIdx.x * 256 + threadIdx.x; e < n; e += gridDim.x * 256) {
    const int r = e / cols, c = e - r * cols;
    dx[(size_t)r * ldx + c] = y[(size_t)r * ldy + c] > 0.f ? dy[(size_t)r * ldd + c] : 0.f;
  }
}

void launch_relu_grad2d(const float* dy, int ldd, const float* y, int ldy, int rows, int cols, float* dx,
                        int ldx, hipStream_t s) {
  const int n = rows * cols;
  if (n <= 0) return;
  hipLaunchKernelGGL(relu_grad2d_kernel, dim3(std::min(8192, cdiv(n, 256))), dim3(256), 0, s, dy, ldd, y,
                     ldy, rows, cols, dx, ldx);
}

// ------------------------------------------------------------ minibatch map
// Frames of a minibatch are packed time-major: step t holds the first
// active(t) envs of the length-sorted env list.  For frame f: src[f] = t*N + env,
// w[f] = 1/(nb T_env), msk[f] = mask at (t, env); env_row[j] = env of row j.
__global__ void __launch_bounds__(256) frame_map_kernel(MapArgs m, const float* __restrict__ mask,
                                                        int32_t* __restrict__ src, float* __restrict__ w,
                                                        float* __restrict__ msk,
                                                        int32_t* __restrict__ env_row) {
  const int f = blockIdx.x * 256 + threadIdx.x;
  if (f < m.nb) env_row[f] = m.env[f];
  if (f >= m.F) return;
  int t = 0, off = 0;
  while (true) {
    int act = 0;
    for (int j = 0; j < m.nb; ++j) act += (m.len[j] > t);
    if (f < off + act) {
      const int j = f - off;
      const int s = t * m.N + m.env[j];
      src[f] = s;
      w[f] = 1.0f / ((float)m.nb * (float)m.len[j]);
      msk[f] = mask[s];
      return;
    }
    off += act;
    ++t;
  }
}

void launch_frame_map(const MapArgs& m, const float* mask, int32_t* src, float* w, float* msk,
                      int32_t* env_row, hipStream_t s) {
  const int n = std::max(m.F, m.nb);
  hipLaunchKernelGGL(frame_map_kernel, dim3(cdiv(n, 256)), dim3(256), 0, s, m, mask, src, w, msk,
                     env_row);
}

// dst[l][j][:] = src[l][env_row[j]][:]
__global__ void __launch_bounds__(256) gather_state_kernel(const float* __restrict__ srcs, int L, int N,
                                                           int nb, int H,
                                                           const int32_t* __restrict__ env_row,
                                                           float* __restrict__ dst) {
  const int n = L * nb * H;
  for (int e = blockIdx.x * 256 + threadIdx.x; e < n; e += gridDim.x * 256) {
    const int j = (e / H) % nb, l = e / (nb * H), k = e % H;
    dst[e] = srcs[((size_t)l * N + env_row[j]) * H + k];
  }
}

void launch_gather_state(const float* srcs, int L, int N, int nb, int H, const int32_t* env_row,
                         float* dst, hipStream_t s) {
  const int n = L * nb * H;
  hipLaunchKernelGGL(gather_state_kernel, dim3(std::min(4096, cdiv(n, 256))), dim3(256), 0, s, srcs, L, N,
                     nb, H, env_row, dst);
}

// Copy of a [rows][cols] window between two strided buffers; with a device
// row count, rows >= *active are left as they are.
__global__ void __launch_bounds__(256) copy2d_kernel(const float* __restrict__ s, int lds, int rows,
                                                     int cols, float* __restrict__ d, int ldd,
                                                     const int32_t* __restrict__ active) {
  if (active) rows = min(rows, max(*active, 0));
  const int n = rows * cols;
  for (int e = blockIdx.x * 256 + threadIdx.x; e < n; e += gridDim.x * 256) {
    const int r = e / cols, c = e - r * cols;
    d[(size_t)r * ldd + c] = s[(size_t)r * lds + c];
  }
}

void launch_copy2d(const float* s_, int lds, int rows, int cols, float* d, int ldd, hipStream_t s,
                   const int32_t* active) {
  const int n = rows * cols;
  if (n <= 0) return;
  hipLaunchKernelGGL(copy2d_kernel, dim3(std::min(4096, cdiv(n, 256))), dim3(256), 0, s, s_, lds, rows,
                     cols, d, ldd, active);
}

// Gradient at a 3-vector goal input: dgoal[f][i] = sum_k dZ[f][zoff + k] gw[k][i]
// (packed frame order).
__global__ void __launch_bounds__(256) goal_dgrad_kernel(const float* __restrict__ dZ, int ldz, int zoff, int F,
                                                         int goal_dim, const float* __restrict__ gw,
                                                         float* __restrict__ dgoal) {
  for (int e = blockIdx.x * 256 + threadIdx.x; e < F * 3; e += gridDim.x * 256) {
    const int f = e / 3, i = e - f * 3;
    const float* dz = dZ + (size_t)f * ldz + zoff;
    float acc = 0.f;
    for (int k = 0; k < goal_dim; ++k) acc = fmaf(dz[k], gw[k * 3 + i], acc);
    dgoal[e] = acc;
  }
}

void launch_goal_dgrad(const float* dZ, int ldz, int zoff, int F, int goal_dim, const float* gw, float* dgoal,
                       hipStream_t s) {
  if (F <= 0) return;
  hipLaunchKernelGGL(goal_dgrad_kernel, dim3(std::min(4096, cdiv(F * 3, 256))), dim3(256), 0, s, dZ, ldz, zoff, F,
                     goal_dim, gw, dgoal);
}

// The planner's PointGoal from its raw head outputs (magnitude ELU(r0) + 0.75,
// direction tanh(r1), tanh(r2)): row f of raw (stride ldr) -> row dst[f] of goal.
__global__ void __launch_bounds__(256) planner_goal_kernel(const float* __restrict__ raw, int ldr,
                                                           const int32_t* __restrict__ dst, int F,
                                                           float* __restrict__ goal) {
  for (int e = blockIdx.x * 256 + threadIdx.x; e < F * 3; e += gridDim.x * 256) {
    const int f = e / 3, i = e - f * 3;
    const float r = raw[(size_t)f * ldr + i];
    const float g = i == 0 ? (r > 0.f ? r : expm1f(r)) + 0.75f : tanhf(r);
    goal[(size_t)(dst ? dst[f] : f) * 3 + i] = g;
  }
}

// draw = dgoal * d goal / d raw (both [F][3], raw rows of stride ldr)
__global__ void __launch_bounds__(256) planner_goal_bwd_kernel(const float* __restrict__ raw, int ldr,
                                                               const float* __restrict__ dgoal, int F,
                                                               float* __restrict__ draw) {
  for (int e = blockIdx.x * 256 + threadIdx.x; e < F * 3; e += gridDim.x * 256) {
    const int f = e / 3, i = e - f * 3;
    const float r = raw[(size_t)f * ldr + i];
    float d;
    if (i == 0) d = r > 0.f ? 1.f : expf(r);
    else {
      const float t = tanhf(r);
      d = 1.f - t * t;
    }
    draw[(size_t)f * ldr + i] = dgoal[e] * d;
  }
}

void launch_planner_goal(const float* raw, int ldr, const int32_t* dst, int F, float* goal, hipStream_t s) {
  if (F <= 0) return;
  hipLaunchKernelGGL(planner_goal_kernel, dim3(std::min(4096, cdiv(F * 3, 256))), dim3(256), 0, s, raw, ldr, dst, F,
                     goal);
}

void launch_planner_goal_bwd(const float* raw, int ldr, const float* dgoal, int F, float* draw, hipStream_t s) {
  if (F <= 0) return;
  hipLaunchKernelGGL(planner_goal_bwd_kernel, dim3(std::min(4096, cdiv(F * 3, 256))), dim3(256), 0, s, raw, ldr,
                     dgoal, F, draw);
}

// Policy/value head over frames: logits[f][k], values[f] (one wavefront per frame).
__global__ void __launch_bounds__(256) head_fwd_kernel(const float* __restrict__ htop, int F, int H, int A,
                                                       const float* __restrict__ W, const float* __restrict__ b,
                                                       float* __restrict__ logits, float* __restrict__ values) {
  const int f = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (f >= F) return;
  float o[kMaxA];
  head_dots(htop + (size_t)f * H, W, b, H, A + 1, o);
  if (lane == 0) {
    for (int k = 0; k < A; ++k) logits[(size_t)f * A + k] = o[k];
    values[f] = o[A];
  }
}

// dout[f] = [dlogits[f], dvalues[f]], dh[f] = dout[f] W.
__global__ void __launch_bounds__(256) head_bwd_kernel(const float* __restrict__ dlogits,
                                                       const float* __restrict__ dvalues, int F, int H, int A,
                                                       const float* __restrict__ W, float* __restrict__ dout,
                                                       float* __restrict__ dh) {
  const int f = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (f >= F) return;
  float d[kMaxA];
#pragma unroll
  for (int k = 0; k < kMaxA; ++k) d[k] = 0.f;
  for (int k = 0; k < A; ++k) d[k] = dlogits[(size_t)f * A + k];
  d[A] = dvalues[f];
  if (lane == 0)
    for (int k = 0; k <= A; ++k) dout[(size_t)f * (A + 1) + k] = d[k];
  head_dh(d, W, H, A + 1, dh + (size_t)f * H);
}

__global__ void __launch_bounds__(256) copy_i32_kernel(const int32_t* __restrict__ s, int n, int32_t* __restrict__ d) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) d[i] = s[i];
}

void launch_head_fwd(const float* htop, int F, int H, int A, const float* W, const float* b, float* logits,
                     float* values, hipStream_t s) {
  hipLaunchKernelGGL(head_fwd_kernel, dim3(cdiv(F, 4)), dim3(256), 0, s, htop, F, H, A, W, b, logits, values);
}

void launch_head_bwd(const float* dlogits, const float* dvalues, int F, int H, int A, const float* W, float* dout,
                     float* dh, hipStream_t s) {
  hipLaunchKernelGGL(head_bwd_kernel, dim3(cdiv(F, 4)), dim3(256), 0, s, dlogits, dvalues, F, H, A, W, dout, dh);
}

void launch_copy_i32(const int32_t* src, int n, int32_t* dst, hipStream_t s) {
  hipLaunchKernelGGL(copy_i32_kernel, dim3(cdiv(n, 256)), dim3(256), 0, s, src, n, dst);
}
