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

// 8 consecutive values as floats: two 16-byte loads (float) or one (bfloat16)
DEV void act_ld8(const float* p, float v[8]) {
  const float4 a = *(const float4*)p, b = *(const float4*)(p + 4);
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}
DEV void act_ld8(const bf16_t* p, float v[8]) {
  const uint4 a = *(const uint4*)p;
  const uint32_t w4[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    v[2 * i] = __uint_as_float(w4[i] << 16);
    v[2 * i + 1] = __uint_as_float(w4[i] & 0xffff0000u);
  }
}

// V8 = false: thread s of a gate column holds k = s + TPC i (i < KMAX), one
// element per load.  V8 = true (din, H, ldx, ldw multiples of 8, operands
// 16-byte aligned): it holds the 8-element chunks c = s + TPC i (i < KMAX)
// of k, one or two 16-byte loads per chunk.
template <typename TW, int U, int KMAX, bool V8>
__global__ void __launch_bounds__(256) lstm_act_layer_kernel(const float* __restrict__ X, int ldx, int din,
                                                             const float* __restrict__ HM,
                                                             const float* __restrict__ CM, const TW* __restrict__ W,
                                                             int ldw, const float* __restrict__ bias, int B, int H,
                                                             float* __restrict__ h_out, float* __restrict__ c_out,
                                                             const int32_t* __restrict__ active) {
  extern __shared__ float gates[];  // [B][4U]
  constexpr int TPC = 64 / U;
  constexpr int E = V8 ? 8 : 1;  // elements per chunk
  constexpr bool BF = sizeof(TW) == 2;
  const int K = din + H, KC = K / E;  // chunks (V8: K % 8 == 0)
  const int j0 = blockIdx.x * U;
  const int col = threadIdx.x / TPC, s = threadIdx.x % TPC;
  const int q = col / U, uc = col % U;
  float w[KMAX][E];
  {
    const TW* wr = W + (size_t)(q * H + j0 + uc) * ldw;
    // unconditional loads (a chunk past K re-reads the last one, then zeroed):
    // a load inside a branch would wait for its own result before the next is issued
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
      const int c = s + TPC * i;
      if constexpr (V8) {
        act_ld8(wr + (size_t)min(c, KC - 1) * 8, w[i]);
      } else {
        w[i][0] = ldf(wr + min(c, K - 1));
      }
#pragma unroll
      for (int e = 0; e < E; ++e) w[i][e] = c < KC ? w[i][e] : 0.f;
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
  auto load_row = [&](int r, float (&v)[KMAX][E]) {
    const float* xr = X + (size_t)r * ldx;
    const float* hr = HM + (size_t)r * H;
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
      const int k = min(s + TPC * i, KC - 1) * E;
      const float* p = k < din ? xr + k : hr + min(k - din, H - E);
      if constexpr (V8)
        act_ld8(p, v[i]);
      else
        v[i][0] = *p;
    }
  };
  float xv[KMAX][E], xn[KMAX][E];
  load_row(0, xv);
  for (int r = 0; r < B; ++r) {
    load_row(min(r + 1, B - 1), xn);
    float acc = 0.f;
#pragma unroll
    for (int i = 0; i < KMAX; ++i)
#pragma unroll
      for (int e = 0; e < E; ++e) acc = fmaf(op_round(xv[i][e], BF), w[i][e], acc);
#pragma unroll
    for (int o = TPC / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
    if (s == 0) gates[r * 4 * U + col] = acc;
#pragma unroll
    for (int i = 0; i < KMAX; ++i)
#pragma unroll
      for (int e = 0; e < E; ++e) xv[i][e] = xn[i][e];
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
    case 8: return (const void*)lstm_act_layer_kernel<TW, U, 8, false>;
    case 16: return (const void*)lstm_act_layer_kernel<TW, U, 16, false>;
    case 32: return (const void*)lstm_act_layer_kernel<TW, U, 32, false>;
    case 64: return (const void*)lstm_act_layer_kernel<TW, U, 64, false>;
    default: return nullptr;
  }
}
// chunks of 8 per thread
template <typename TW, int U>
const void* act_kernel_v8(int kc) {
  switch (kc) {
    case 1: return (const void*)lstm_act_layer_kernel<TW, U, 1, true>;
    case 2: return (const void*)lstm_act_layer_kernel<TW, U, 2, true>;
    case 3: return (const void*)lstm_act_layer_kernel<TW, U, 3, true>;
    case 4: return (const void*)lstm_act_layer_kernel<TW, U, 4, true>;
    case 5: return (const void*)lstm_act_layer_kernel<TW, U, 5, true>;
    case 6: return (const void*)lstm_act_layer_kernel<TW, U, 6, true>;
    case 8: return (const void*)lstm_act_layer_kernel<TW, U, 8, true>;
    default: return nullptr;
  }
}
int v8_chunks(int K, int U) {
  const int kc = cdiv(K / 8, 64 / U);
  return kc <= 6 ? kc : kc <= 8 ? 8 : 0;
}
bool v8_ok(const float* X, int ldx, int din, const float* HM, const void* W, int ldw, int H) {
  return din % 8 == 0 && H % 8 == 0 && ldx % 8 == 0 && ldw % 8 == 0 && ((uintptr_t)X & 15) == 0 &&
         ((uintptr_t)HM & 15) == 0 && ((uintptr_t)W & 15) == 0;
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
  const void* k = nullptr;
  const int kc = v8_chunks(din + H, U);
  if (kc && v8_ok(X, ldx, din, HM, W, ldw, H)) {
    if (prec == 1) k = U == 2 ? act_kernel_v8<bf16_t, 2>(kc) : act_kernel_v8<bf16_t, 1>(kc);
    else k = U == 2 ? act_kernel_v8<float, 2>(kc) : act_kernel_v8<float, 1>(kc);
  } else {
    const int kpt = cdiv(din + H, 64 / U);
    const int kmax = kpt <= 8 ? 8 : kpt <= 16 ? 16 : kpt <= 32 ? 32 : 64;
    if (prec == 1) k = U == 2 ? act_kernel_k<bf16_t, 2>(kmax) : act_kernel_k<bf16_t, 1>(kmax);
    else k = U == 2 ? act_kernel_k<float, 2>(kmax) : act_kernel_k<float, 1>(kmax);
  }
  const size_t shmem = (size_t)B * 4 * U * sizeof(float);
  void* args[] = {(void*)&X, (void*)&ldx, (void*)&din, (void*)&HM, (void*)&CM, (void*)&W, (void*)&ldw,
                  (void*)&bias, (void*)&B, (void*)&H, (void*)&h_out, (void*)&c_out, (void*)&active};
  hipLaunchKernel(k, dim3(H / U), dim3(256), args, shmem, s);
}
