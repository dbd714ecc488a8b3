// LSTM cell pointwise kernels (gate order i, f, g, o; float32 state).
// The gate pre-activations come from the MFMA GEMMs; these kernels apply the
// nonlinearities, update c and h, and write the episode-masked state that
// the next step consumes (h, c <- m_{t+1} h, m_{t+1} c).
#include "common.h"
#include "kernels.h"

// G [rows][4H]: pre-activations in, activations (sigma i, sigma f, tanh g,
// sigma o) out.  cp [rows][H]: masked previous c.  h, c [rows][H] out.
// hp_next/cp_next [rows_next][H] = mask_next * (h, c) for rows < rows_next.
__global__ void __launch_bounds__(256) lstm_fwd_kernel(float* __restrict__ G, const float* __restrict__ cp,
                                                       float* __restrict__ h, int ldh, float* __restrict__ c,
                                                       int rows, int H, const float* __restrict__ mask_next,
                                                       int rows_next, float* __restrict__ hp_next,
                                                       float* __restrict__ cp_next) {
  const int n = rows * H;
  for (int e = blockIdx.x * 256 + threadIdx.x; e < n; e += gridDim.x * 256) {
    const int r = e / H, j = e - r * H;
    float* g = G + (size_t)r * 4 * H;
    const float ig = sigm(g[j]);
    const float fg = sigm(g[H + j]);
    const float gg = tanhf(g[2 * H + j]);
    const float og = sigm(g[3 * H + j]);
    const float c2 = fg * cp[e] + ig * gg;
    const float h2 = og * tanhf(c2);
    g[j] = ig;
    g[H + j] = fg;
    g[2 * H + j] = gg;
    g[3 * H + j] = og;
    c[e] = c2;
    h[(size_t)r * ldh + j] = h2;
    if (r < rows_next && hp_next) {
      const float m = mask_next[r];
      hp_next[e] = m * h2;
      cp_next[e] = m * c2;
    }
  }
}

// hp = mask * h_in, cp = mask * c_in  ([rows][H]); hp row stride ldhp.
__global__ void __launch_bounds__(256) mask_state_kernel(const float* __restrict__ h_in,
                                                         const float* __restrict__ c_in,
                                                         const float* __restrict__ mask, int rows, int H,
                                                         float* __restrict__ hp, int ldhp,
                                                         float* __restrict__ cp) {
  const int n = rows * H;
  for (int e = blockIdx.x * 256 + threadIdx.x; e < n; e += gridDim.x * 256) {
    const int r = e / H, j = e - r * H;
    const float m = mask[r];
    hp[(size_t)r * ldhp + j] = m * h_in[e];
    cp[e] = m * c_in[e];
  }
}

// Backward of one step.  act [rows][4H] activations, c [rows][H] = c_t,
// cp [rows][H] = masked c_{t-1}, dh_in [rows][ldd] from above.  Carried
// gradients from step t+1 (rows < rows_next): dh += mask_next * dhp_next,
// dc += mask_next * dcp_next.  Writes dG [rows][4H] (pre-activation) and
// dcp [rows][H] = dc * f.
__global__ void __launch_bounds__(256) lstm_bwd_kernel(const float* __restrict__ act,
                                                       const float* __restrict__ c,
                                                       const float* __restrict__ cp,
                                                       const float* __restrict__ dh_in, int ldd, int rows,
                                                       int H, const float* __restrict__ mask_next,
                                                       int rows_next, const float* __restrict__ dhp_next,
                                                       const float* __restrict__ dcp_next,
                                                       float* __restrict__ dG, float* __restrict__ dcp) {
  const int n = rows * H;
  for (int e = blockIdx.x * 256 + threadIdx.x; e < n; e += gridDim.x * 256) {
    const int r = e / H, j = e - r * H;
    const float* a = act + (size_t)r * 4 * H;
    const float ig = a[j], fg = a[H + j], gg = a[2 * H + j], og = a[3 * H + j];
    float dh = dh_in[(size_t)r * ldd + j];
    float dc = 0.f;
    if (r < rows_next && dhp_next) {
      const float m = mask_next[r];
      dh += m * dhp_next[e];
      dc += m * dcp_next[e];
    }
    const float tc = tanhf(c[e]);
    const float d_o = dh * tc;
    dc += dh * og * (1.f - tc * tc);
    const float d_i = dc * gg, d_g = dc * ig, d_f = dc * cp[e];
    float* d = dG + (size_t)r * 4 * H;
    d[j] = d_i * ig * (1.f - ig);
    d[H + j] = d_f * fg * (1.f - fg);
    d[2 * H + j] = d_g * (1.f - gg * gg);
    d[3 * H + j] = d_o * og * (1.f - og);
    dcp[e] = dc * fg;
  }
}

// out[n] = alpha * sum_r in[r*ld + n] for r < rows (fixed order; one thread per column)
__global__ void __launch_bounds__(256) colsum_kernel(const float* __restrict__ in, int rows, int cols,
                                                     int ld, float* __restrict__ out) {
  const int n = blockIdx.x * 256 + threadIdx.x;
  if (n >= cols) return;
  float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
  int r = 0;
  for (; r + 4 <= rows; r += 4) {
    s0 += in[(size_t)r * ld + n];
    s1 += in[(size_t)(r + 1) * ld + n];
    s2 += in[(size_t)(r + 2) * ld + n];
    s3 += in[(size_t)(r + 3) * ld + n];
  }
  for (; r < rows; ++r) s0 += in[(size_t)r * ld + n];
  out[n] = (s0 + s1) + (s2 + s3);
}

void launch_lstm_fwd(float* G, const float* cp, float* h, int ldh, float* c, int rows, int H,
                     const float* mask_next, int rows_next, float* hp_next, float* cp_next,
                     hipStream_t s) {
  const int n = rows * H;
  if (n <= 0) return;
  hipLaunchKernelGGL(lstm_fwd_kernel, dim3(std::min(4096, cdiv(n, 256))), dim3(256), 0, s, G, cp, h, ldh,
                     c, rows, H, mask_next, rows_next, hp_next, cp_next);
}

void launch_mask_state(const float* h_in, const float* c_in, const float* mask, int rows, int H,
                       float* hp, int ldhp, float* cp, hipStream_t s) {
  const int n = rows * H;
  if (n <= 0) return;
  hipLaunchKernelGGL(mask_state_kernel, dim3(std::min(4096, cdiv(n, 256))), dim3(256), 0, s, h_in, c_in,
                     mask, rows, H, hp, ldhp, cp);
}

void launch_lstm_bwd(const float* act, const float* c, const float* cp, const float* dh_in, int ldd,
                     int rows, int H, const float* mask_next, int rows_next, const float* dhp_next,
                     const float* dcp_next, float* dG, float* dcp, hipStream_t s) {
  const int n = rows * H;
  if (n <= 0) return;
  hipLaunchKernelGGL(lstm_bwd_kernel, dim3(std::min(4096, cdiv(n, 256))), dim3(256), 0, s, act, c, cp,
                     dh_in, ldd, rows, H, mask_next, rows_next, dhp_next, dcp_next, dG, dcp);
}

void launch_colsum(const float* in, int rows, int cols, int ld, float* out, hipStream_t s) {
  hipLaunchKernelGGL(colsum_kernel, dim3(cdiv(cols, 256)), dim3(256), 0, s, in, rows, cols, ld, out);
}
