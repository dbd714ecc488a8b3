// Fused LSTM time steps: one launch per step and direction.
//
// Forward step: gates = G_in + X W^T (+ b) for a 32-row x (4 gates x 8 units)
// block, then the cell pointwise (i, f, o sigmoid, g tanh; c = f c_prev + i g,
// h = o tanh c) and the episode-masked state of the next step.  Backward step:
// dHP_{t+1} = dG_{t+1} W_hh for a 32-row x 8-unit block (W_hh^T is copied
// once per call so these reads are contiguous), then the pointwise backward
// of step t for those units.  The small products use MFMAs whose operands
// are read straight from global memory (the recurrent weights and the step's
// rows are L2 resident), several k-steps in flight; each of the 4
// wavefronts takes a quarter of K and the partial tiles are summed in LDS.
#include "gemm.h"
#include "kernels.h"

namespace {

// A(m, k) = a[m*am + k*ak]; 8 consecutive k of row m (0 outside [0,M) x [0,K)).
template <typename T>
DEV void row8(const T* a, int am, int ak, int m, int M, int k, int K, float v[8]) {
  if (m >= M) return zero8(v);
  const T* p = a + (size_t)m * am + (size_t)k * ak;
  if (ak == 1 && k + 8 <= K && aligned16(p)) return load8(p, v);
#pragma unroll
  for (int e = 0; e < 8; ++e) v[e] = (k + e < K) ? ldf(p + (size_t)e * ak) : 0.f;
}

template <typename TC>
DEV void to_op(const float v[8], TC* hi, TC* lo, bool split);
template <>
DEV void to_op<float>(const float v[8], float* hi, float*, bool) {
#pragma unroll
  for (int e = 0; e < 8; ++e) hi[e] = v[e];
}
template <>
DEV void to_op<bf16_t>(const float v[8], bf16_t* hi, bf16_t* lo, bool split) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    hi[e] = f2bf(v[e]);
    lo[e] = split ? f2bf(v[e] - bf2f(hi[e])) : (bf16_t)0;
  }
}

// The 4 wavefronts split [0, K) into multiples of 16.
DEV void wave_krange(int K, int& k0, int& k1) {
  const int w = threadIdx.x >> 6;
  const int steps = (K + 15) / 16;
  const int per = (steps + 3) / 4;
  k0 = min(K, w * per * 16);
  k1 = min(K, (w + 1) * per * 16);
}

// One wavefront's 32x32 tile over k in [k0, k1): A rows from `a` (row stride
// lda, contiguous k), B column n from brow(n) (contiguous k).  Operands for 8
// k-steps are loaded before their MFMAs so the loads overlap.
template <typename TC, typename TB, bool SPLIT, class BRow>
DEV void wave_tile_pf(const float* a, int lda, int M, BRow brow, int N, int k0, int k1, float* red) {
  using MM = Mma<TC>;
  constexpr int FR = MM::FR;
  constexpr int F = 32 / FR;
  constexpr int PF = 8 / (2 * F);  // k-steps in flight: 4 (bfloat16) or 2 (float32)
  const int lane = threadIdx.x & 63;
  typename MM::Acc acc[F][F];
#pragma unroll
  for (int i = 0; i < F; ++i)
#pragma unroll
    for (int j = 0; j < F; ++j) acc[i][j] = MM::zero();
  for (int kb = k0; kb < k1; kb += 16 * PF) {
    float va[PF][F][8], vb[PF][F][8];
#pragma unroll
    for (int st = 0; st < PF; ++st) {
      const int kk = kb + st * 16 + MM::kof(lane);
#pragma unroll
      for (int i = 0; i < F; ++i) {
        const int r = i * FR + MM::row(lane);
        row8(a, lda, 1, r, M, kk, k1, va[st][i]);
        const TB* bp = brow(r);
        if (r < N) row8(bp, 0, 1, 0, 1, kk, k1, vb[st][i]);
        else zero8(vb[st][i]);
      }
    }
#pragma unroll
    for (int st = 0; st < PF; ++st) {
      if (kb + st * 16 >= k1) break;
      __attribute__((aligned(16))) TC ah[F][8], al[F][8], bh[F][8], bl[F][8];
#pragma unroll
      for (int i = 0; i < F; ++i) {
        to_op<TC>(va[st][i], ah[i], al[i], SPLIT);
        to_op<TC>(vb[st][i], bh[i], bl[i], false);
      }
#pragma unroll
      for (int i = 0; i < F; ++i)
#pragma unroll
        for (int j = 0; j < F; ++j) {
          acc[i][j] = MM::mma(ah[i], bh[j], acc[i][j]);
          if (SPLIT) acc[i][j] = MM::mma(al[i], bh[j], acc[i][j]);
        }
    }
  }
#pragma unroll
  for (int i = 0; i < F; ++i)
#pragma unroll
    for (int j = 0; j < F; ++j)
#pragma unroll
      for (int r = 0; r < MM::NOUT; ++r)
        red[(i * FR + MM::orow(lane, r)) * 33 + j * FR + MM::ocol(lane)] = acc[i][j][r];
}

template <typename TC, typename TW>
__global__ void __launch_bounds__(256) lstm_step_fwd_kernel(
    const float* __restrict__ X, int ldx, int K, const TW* __restrict__ W, int ldw,
    const float* __restrict__ Gin, const float* __restrict__ bias, const float* __restrict__ cprev,
    int rows, int H, float* __restrict__ act, float* __restrict__ h_out, int ldh, float* __restrict__ c_out,
    const float* __restrict__ mask_next, int rows_next, float* __restrict__ hp_next, int ldhp,
    float* __restrict__ cp_next) {
  __shared__ float red[4][32 * 33];
  const int j0 = blockIdx.x * 8, r0 = blockIdx.y * 32;
  int k0, k1;
  wave_krange(K, k0, k1);
  // gate column n (0..31) <-> weight row (n/8)*H + j0 + n%8
  auto brow = [&](int n) { return W + (size_t)((n >> 3) * H + j0 + (n & 7)) * ldw; };
  wave_tile_pf<TC, TW, false>(X + (size_t)r0 * ldx, ldx, rows - r0, brow, 32, k0, k1, red[threadIdx.x >> 6]);
  __syncthreads();
  const int row = threadIdx.x >> 3, u = threadIdx.x & 7;
  const int r = r0 + row, j = j0 + u;
  if (r >= rows || j >= H) return;
  float pre[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int col = q * 8 + u;
    float s = red[0][row * 33 + col] + red[1][row * 33 + col] + red[2][row * 33 + col] +
              red[3][row * 33 + col];
    if (Gin) s += Gin[(size_t)r * 4 * H + q * H + j];
    if (bias) s += bias[q * H + j];
    pre[q] = s;
  }
  const float ig = sigm(pre[0]), fg = sigm(pre[1]), gg = tanhf(pre[2]), og = sigm(pre[3]);
  const float c2 = fg * cprev[(size_t)r * H + j] + ig * gg;
  const float h2 = og * tanhf(c2);
  if (act) {
    float* a = act + (size_t)r * 4 * H;
    a[j] = ig;
    a[H + j] = fg;
    a[2 * H + j] = gg;
    a[3 * H + j] = og;
  }
  c_out[(size_t)r * H + j] = c2;
  h_out[(size_t)r * ldh + j] = h2;
  if (hp_next && r < rows_next) {
    const float m = mask_next[r];
    hp_next[(size_t)r * ldhp + j] = m * h2;
    cp_next[(size_t)r * H + j] = m * c2;
  }
}

// Backward of step t for 8 units x 32 rows.  With dGn (= dG_{t+1}, rows_n
// rows) first dHP = dGn W_hh for these units (W_hh^T given as WT [H][4H]);
// then dh = dH_in + m_{t+1} dHP, dc = m_{t+1} dcp (rows < rows_n) and the
// cell's pointwise backward -> dG_t, dcp_t (dcp updated in place).
template <typename TC, typename TW, bool SPLIT>
__global__ void __launch_bounds__(256) lstm_step_bwd_kernel(
    const float* __restrict__ dGn, const TW* __restrict__ WT, const float* __restrict__ mask_n, int rows_n,
    const float* __restrict__ act, const float* __restrict__ c, const float* __restrict__ cp,
    const float* __restrict__ dH, int ldd, int rows, int H, float* __restrict__ dG, float* __restrict__ dcp) {
  __shared__ float red[4][32 * 33];
  const int j0 = blockIdx.x * 8, r0 = blockIdx.y * 32;
  const bool carry = dGn != nullptr && r0 < rows_n;
  if (carry) {
    int k0, k1;
    wave_krange(4 * H, k0, k1);
    auto brow = [&](int n) { return WT + (size_t)(j0 + n) * 4 * H; };
    wave_tile_pf<TC, TW, SPLIT>(dGn + (size_t)r0 * 4 * H, 4 * H, rows_n - r0, brow, min(8, H - j0), k0, k1,
                                red[threadIdx.x >> 6]);
  }
  __syncthreads();
  const int row = threadIdx.x >> 3, u = threadIdx.x & 7;
  const int r = r0 + row, j = j0 + u;
  if (r >= rows || j >= H) return;
  float dh = dH[(size_t)r * ldd + j];
  float dc = 0.f;
  if (carry && r < rows_n) {
    const float m = mask_n[r];
    const float s = red[0][row * 33 + u] + red[1][row * 33 + u] + red[2][row * 33 + u] + red[3][row * 33 + u];
    dh += m * s;
    dc = m * dcp[(size_t)r * H + j];
  }
  const float* a = act + (size_t)r * 4 * H;
  const float ig = a[j], fg = a[H + j], gg = a[2 * H + j], og = a[3 * H + j];
  const float tc = tanhf(c[(size_t)r * H + j]);
  const float d_o = dh * tc;
  dc += dh * og * (1.f - tc * tc);
  float* d = dG + (size_t)r * 4 * H;
  d[j] = dc * gg * ig * (1.f - ig);
  d[H + j] = dc * cp[(size_t)r * H + j] * fg * (1.f - fg);
  d[2 * H + j] = dc * ig * (1.f - gg * gg);
  d[3 * H + j] = d_o * og * (1.f - og);
  dcp[(size_t)r * H + j] = dc * fg;
}

// WT[j][g] = W[g][j] for g < 4H, j < H (W row stride ldw).
template <typename TW>
__global__ void __launch_bounds__(256) transpose_whh_kernel(const TW* __restrict__ W, int ldw, int H,
                                                            TW* __restrict__ WT) {
  __shared__ TW tile[32][33];
  const int g0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int y = ty; y < 32; y += 8)
    if (g0 + y < 4 * H && j0 + tx < H) tile[y][tx] = W[(size_t)(g0 + y) * ldw + j0 + tx];
  __syncthreads();
  for (int y = ty; y < 32; y += 8)
    if (j0 + y < H && g0 + tx < 4 * H) WT[(size_t)(j0 + y) * 4 * H + g0 + tx] = tile[tx][y];
}

}  // namespace

void launch_lstm_step_fwd(int prec, const float* X, int ldx, int K, const void* W, int ldw, const float* Gin,
                          const float* bias, const float* cprev, int rows, int H, float* act, float* h_out,
                          int ldh, float* c_out, const float* mask_next, int rows_next, float* hp_next,
                          int ldhp, float* cp_next, hipStream_t s) {
  if (rows <= 0) return;
  const dim3 grid(cdiv(H, 8), cdiv(rows, 32));
  if (prec == 1)
    hipLaunchKernelGGL((lstm_step_fwd_kernel<bf16_t, bf16_t>), grid, dim3(256), 0, s, X, ldx, K,
                       (const bf16_t*)W, ldw, Gin, bias, cprev, rows, H, act, h_out, ldh, c_out, mask_next,
                       rows_next, hp_next, ldhp, cp_next);
  else
    hipLaunchKernelGGL((lstm_step_fwd_kernel<float, float>), grid, dim3(256), 0, s, X, ldx, K,
                       (const float*)W, ldw, Gin, bias, cprev, rows, H, act, h_out, ldh, c_out, mask_next,
                       rows_next, hp_next, ldhp, cp_next);
}

void launch_lstm_step_bwd(int prec, const float* dGn, const void* WT, const float* mask_n, int rows_n,
                          const float* act, const float* c, const float* cp, const float* dH, int ldd, int rows,
                          int H, float* dG, float* dcp, hipStream_t s) {
  if (rows <= 0) return;
  const dim3 grid(cdiv(H, 8), cdiv(rows, 32));
  if (prec == 1)
    hipLaunchKernelGGL((lstm_step_bwd_kernel<bf16_t, bf16_t, true>), grid, dim3(256), 0, s, dGn,
                       (const bf16_t*)WT, mask_n, rows_n, act, c, cp, dH, ldd, rows, H, dG, dcp);
  else
    hipLaunchKernelGGL((lstm_step_bwd_kernel<float, float, false>), grid, dim3(256), 0, s, dGn,
                       (const float*)WT, mask_n, rows_n, act, c, cp, dH, ldd, rows, H, dG, dcp);
}

void launch_transpose_whh(int prec, const void* W, int ldw, int H, void* WT, hipStream_t s) {
  const dim3 grid(cdiv(4 * H, 32), cdiv(H, 32));
  if (prec == 1)
    hipLaunchKernelGGL(transpose_whh_kernel<bf16_t>, grid, dim3(256), 0, s, (const bf16_t*)W, ldw, H, (bf16_t*)WT);
  else
    hipLaunchKernelGGL(transpose_whh_kernel<float>, grid, dim3(256), 0, s, (const float*)W, ldw, H, (float*)WT);
}
