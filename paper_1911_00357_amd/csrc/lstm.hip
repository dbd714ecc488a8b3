// Small helpers of the recurrent core: the episode-masked start state of a
// minibatch (h, c <- m h, m c) and the column sums that give bias gradients.
#include "common.h"
#include "kernels.h"

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

void launch_mask_state(const float* h_in, const float* c_in, const float* mask, int rows, int H,
                       float* hp, int ldhp, float* cp, hipStream_t s) {
  const int n = rows * H;
  if (n <= 0) return;
  hipLaunchKernelGGL(mask_state_kernel, dim3(std::min(4096, cdiv(n, 256))), dim3(256), 0, s, h_in, c_in,
                     mask, rows, H, hp, ldhp, cp);
}

void launch_colsum(const float* in, int rows, int cols, int ld, float* out, hipStream_t s) {
  hipLaunchKernelGGL(colsum_kernel, dim3(cdiv(cols, 256)), dim3(256), 0, s, in, rows, cols, ld, out);
}
