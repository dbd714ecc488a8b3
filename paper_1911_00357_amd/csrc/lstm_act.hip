// The act step's recurrent core (Sec. 4 "Agent"; App. "Agent Design": goal
// encoder, previous-action embedding, 2-layer LSTM) for one time step of a
// small batch of envs, in L + 1 launches:
//
//   act_core_prep_kernel   goal FC / raw goal and the previous-action
//                          embedding into the layer-0 input rows, and the
//                          episode-masked copies m h, m c of every layer's
//                          state (all read before any layer writes its
//                          output, so h_out / c_out may alias h_in / c_in);
//   lstm_act_layer_kernel  one layer: gates = [x | m h] [W_ih | W_hh]^T + b
//                          and the cell, per workgroup for U hidden units;
//                          with a device row count, only the rows below it
//                          are written.
//
// The layer kernel keeps its 4U weight rows in registers (lane s of a gate
// column holds k = s + TPC*i) and forms each gate with FMAs and a lane
// reduction; with bfloat16 weights the operands are rounded to bfloat16 as
// the matrix-core path does, products are exact in float32.
#include "common.h"
#include "kernels.h"

namespace {

__global__ void __launch_bounds__(256) act_core_prep_kernel(
    const float* __restrict__ goal, const int32_t* __restrict__ prev_a, const float* __restrict__ mask, int B,
    int polar, int goal_dim, const float* __restrict__ gw, const float* __restrict__ gb, int E,
    const float* __restrict__ emb, float* __restrict__ Z, int ldz, int zoff, const float* __restrict__ h_in,
    const float* __restrict__ c_in, int L, int SR, int H, float* __restrict__ hm, float* __restrict__ cm) {
  const int per = goal_dim + E;
  const int n0 = B * per, n = n0 + L * B * H;
  for (int e = blockIdx.x * 256 + threadIdx.x; e < n; e += gridDim.x * 256) {
    if (e < n0) {
      const int f = e / per, k = e - f * per;
      float v;
      if (k < goal_dim) {
        // goal modes: 0 raw 2-vector, 1 polar (d, theta) -> [d, cos, sin] -> FC, 2 a 3-vector -> FC
        if (polar == 2) {
          const float* g3 = goal + (size_t)f * 3;
          v = gb[k] + gw[k * 3] * g3[0] + gw[k * 3 + 1] * g3[1] + gw[k * 3 + 2] * g3[2];
        } else {
          const float d = goal[(size_t)f * 2], th = goal[(size_t)f * 2 + 1];
          v = polar ? gb[k] + gw[k * 3] * d + gw[k * 3 + 1] * cosf(th) + gw[k * 3 + 2] * sinf(th)
                    : (k == 0 ? d : th);
        }
      } else {
        const int idx = (mask[f] == 0.f) ? 0 : prev_a[f] + 1;
        v = emb[(size_t)idx * E + (k - goal_dim)];
      }
      Z[(size_t)f * ldz + zoff + k] = v;
    } else {
      const int q = e - n0, l = q / (B * H), r = (q - l * B * H) / H, j = q - l * B * H - r * H;
      const float m = mask[r];
      const size_t src = ((size_t)l * SR + r) * H + j;
      hm[(size_t)l * B * H + (size_t)r * H + j] = m * h_in[src];
      cm[(size_t)l * B * H + (size_t)r * H + j] = m * c_in[src];
    }
  }
}

// bfloat16 rounding (round to nearest even) without branches
typedef __bf16 act_bf16x2 __attribute__((ext_vector_type(2)));
typedef float act_f32x2 __attribute__((ext_vector_type(2)));
DEV float op_round(float x, bool bf) {
  if (!bf) return x;
  const act_bf16x2 r = __builtin_convertvector((act_f32x2){x, 0.f}, act_bf16x2);
  return __uint_as_float((uint32_t)__builtin_bit_cast(uint32_t, r) << 16);
}

template <typename TW, int U, int KMAX>
__global__ void __launch_bounds__(256) lstm_act_layer_kernel(const float* __restrict__ X, int ldx, int din,
                                                             const float* __restrict__ HM,
                                                             const float* __restrict__ CM, const TW* __restrict__ W,
                                                             int ldw, const float* __restrict__ bias, int B, int H,
                                                             float* __restrict__ h_out, float* __restrict__ c_out,
                                                             const int32_t* __restrict__ active) {
  extern __shared__ float gates[];  // [B][4U]
  constexpr int TPC = 64 / U;
  constexpr bool BF = sizeof(TW) == 2;
  const int K = din + H;
  const int j0 = blockIdx.x * U;
  const int col = threadIdx.x / TPC, s = threadIdx.x % TPC;
  const int q = col / U, uc = col % U;
  float w[KMAX];
  {
    const TW* wr = W + (size_t)(q * H + j0 + uc) * ldw;
    // unconditional loads (k >= K re-reads element K-1, then zeroed): a load
    // inside a branch would wait for its own result before the next is issued
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
      const int k = s + TPC * i;
      const float t = ldf(wr + min(k, K - 1));
      w[i] = k < K ? t : 0.f;
    }
  }
  // pointwise operands of this thread's first item, loaded before the products
  const int it0 = threadIdx.x, r0 = it0 / U, u0 = it0 - r0 * U, j0p = j0 + u0;
  float pb[4] = {0.f, 0.f, 0.f, 0.f}, pc = 0.f;
  if (it0 < B * U) {
#pragma unroll
    for (int qq = 0; qq < 4; ++qq) pb[qq] = bias[qq * H + j0p];
    pc = CM[(size_t)r0 * H + j0p];
  }
  // every load unconditional (k >= K reads a valid element that meets a zero
  // weight), so all of them are in flight together; row r + 1 is loaded while
  // row r is reduced
  auto load_row = [&](int r, float (&v)[KMAX]) {
    const float* xr = X + (size_t)r * ldx;
    const float* hr = HM + (size_t)r * H;
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
      const int k = s + TPC * i;
      const float* p = k < din ? xr + k : hr + min(k - din, H - 1);
      v[i] = *p;
    }
  };
  float xv[KMAX], xn[KMAX];
  load_row(0, xv);
  for (int r = 0; r < B; ++r) {
    load_row(min(r + 1, B - 1), xn);
    float acc = 0.f;
#pragma unroll
    for (int i = 0; i < KMAX; ++i) acc = fmaf(op_round(xv[i], BF), w[i], acc);
#pragma unroll
    for (int o = TPC / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
    if (s == 0) gates[r * 4 * U + col] = acc;
#pragma unroll
    for (int i = 0; i < KMAX; ++i) xv[i] = xn[i];
  }
  __syncthreads();
  // rows >= *active (a device count, read when the kernel runs) keep their state
  const int nw = active ? min(max(*active, 0), B) : B;
  for (int it = threadIdx.x; it < nw * U; it += 256) {
    const int r = it / U, u = it - r * U, j = j0 + u;
    const float* gr = gates + r * 4 * U + u;
    const bool first = it == it0;
    const float b0 = first ? pb[0] : bias[j], b1 = first ? pb[1] : bias[H + j];
    const float b2 = first ? pb[2] : bias[2 * H + j], b3 = first ? pb[3] : bias[3 * H + j];
    const float ig = sigm(gr[0] + b0), fg = sigm(gr[U] + b1);
    const float gg = tanhf(gr[2 * U] + b2), og = sigm(gr[3 * U] + b3);
    const float c2 = fg * (first ? pc : CM[(size_t)r * H + j]) + ig * gg;
    c_out[(size_t)r * H + j] = c2;
    h_out[(size_t)r * H + j] = og * tanhf(c2);
  }
}

int act_units(int H) { return H >= 512 ? 2 : 1; }

template <typename TW, int U>
const void* act_kernel_k(int kmax) {
  switch (kmax) {
    case 8: return (const void*)lstm_act_layer_kernel<TW, U, 8>;
    case 16: return (const void*)lstm_act_layer_kernel<TW, U, 16>;
    case 32: return (const void*)lstm_act_layer_kernel<TW, U, 32>;
    case 64: return (const void*)lstm_act_layer_kernel<TW, U, 64>;
    default: return nullptr;
  }
}

}  // namespace

void launch_act_core_prep(const float* goal, const int32_t* prev_a, const float* mask, int B, int polar,
                          int goal_dim, const float* gw, const float* gb, int E, const float* emb, float* Z, int ldz,
                          int zoff, const float* h_in, const float* c_in, int L, int SR, int H, float* hm, float* cm,
                          hipStream_t s) {
  const int n = B * (goal_dim + E) + L * B * H;
  if (n <= 0) return;
  hipLaunchKernelGGL(act_core_prep_kernel, dim3(std::min(4096, cdiv(n, 256))), dim3(256), 0, s, goal, prev_a, mask,
                     B, polar, goal_dim, gw, gb, E, emb, Z, ldz, zoff, h_in, c_in, L, SR, H, hm, cm);
}

bool act_layer_supported(int din, int H, int B) {
  const int U = act_units(H);
  if (H % U || H / U > 4096 || B <= 0 || (size_t)B * 4 * U * sizeof(float) > 32768) return false;
  const int kpt = cdiv(din + H, 64 / U);
  return kpt <= 64;
}

void launch_lstm_act_layer(int prec, const float* X, int ldx, int din, const float* HM, const float* CM,
                           const void* W, int ldw, const float* bias, int B, int H, float* h_out, float* c_out,
                           const int32_t* active, hipStream_t s) {
  const int U = act_units(H);
  const int kpt = cdiv(din + H, 64 / U);
  const int kmax = kpt <= 8 ? 8 : kpt <= 16 ? 16 : kpt <= 32 ? 32 : 64;
  const void* k = nullptr;
  if (prec == 1) k = U == 2 ? act_kernel_k<bf16_t, 2>(kmax) : act_kernel_k<bf16_t, 1>(kmax);
  else k = U == 2 ? act_kernel_k<float, 2>(kmax) : act_kernel_k<float, 1>(kmax);
  const size_t shmem = (size_t)B * 4 * U * sizeof(float);
  void* args[] = {(void*)&X, (void*)&ldx, (void*)&din, (void*)&HM, (void*)&CM, (void*)&W, (void*)&ldw,
                  (void*)&bias, (void*)&B, (void*)&H, (void*)&h_out, (void*)&c_out, (void*)&active};
  hipLaunchKernel(k, dim3(H / U), dim3(256), args, shmem, s);
}
