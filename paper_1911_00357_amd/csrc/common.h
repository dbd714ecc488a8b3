// Device helpers shared by the gfx950 kernels of the library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define DEV __device__ __forceinline__

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef uint16_t bf16_t;  // storage type of bfloat16 values

constexpr int kWave = 64;

// float -> bfloat16, round to nearest even (NaN kept quiet).
DEV bf16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (bf16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
}
DEV float bf2f(bf16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

// Loads of a stored element as float, for float or bfloat16 storage.
DEV float ldf(const float* p) { return *p; }
DEV float ldf(const bf16_t* p) { return bf2f(*p); }

DEV float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
DEV double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
DEV float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, kWave));
  return v;
}

DEV float sigmoidf_(float x) { return 1.0f / (1.0f + __expf(-x)); }

// Accurate sigmoid/tanh for the recurrent core (expf, not the fast path).
DEV float sigm(float x) { return 1.0f / (1.0f + expf(-x)); }

inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }
