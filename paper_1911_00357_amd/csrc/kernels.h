// Host-side launchers of the device kernels (all asynchronous on stream s).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <array>
#include <map>
#include <utility>

#include "../../include/ddppo.h"

typedef uint16_t bf16_t;

// Division by a runtime constant as a multiply-high and shift (round-up
// method; exact for 0 <= n < 2^31, d >= 1).
struct FastDiv {
  uint32_t mul, shift;
  __device__ __forceinline__ int div(int n) const {
    return (int)((__umulhi((uint32_t)n, mul) + (uint32_t)n) >> shift);
  }
};
inline FastDiv fast_div(int d) {
  uint32_t s = 0;
  while ((1ull << s) < (uint64_t)d) ++s;
  const uint64_t m = ((1ull << 32) * ((1ull << s) - (uint64_t)d)) / (uint64_t)d + 1;
  return FastDiv{(uint32_t)m, s};
}

// Convolution geometry (NHWC activations, weights [Co][KH][KW][C]).
struct ConvGeo {
  int B, H, W, C;  // input
  int Ho, Wo, Co;  // output
  int KH, KW, stride, pad;
};

// GEMM epilogue: C = alpha * acc (+ C if accumulate) (+ bias[n]) (ReLU).
// Row m of the product is row crow(m) of C: m itself, or (rq > 0) the
// strided map (m / rq) rs1 + ((m % rq) / rwq) rs2 + (m % rwq) rs3 + r0 used
// by the stride-2 data gradient's parity classes.
struct Epi {
  float* C;
  int ldc;
  const float* bias;
  float alpha;
  int relu;
  int accumulate;
  float* partial;  // set by the launcher for split-K
  int rq, rwq, rs1, rs2, rs3, r0;
  // group-major output (gm_p > 0; plain stores only: alpha 1, no bias, ReLU or
  // accumulation): rows m = (image b, pixel p < gm_p), columns n = (group g,
  // channel c < gm_cg) go to ((b G + g) gm_p + p) gm_cg + c, so every (image,
  // group) slab of a GroupNorm is contiguous; split-K partial z at z M N + that
  int gm_p, gm_cg;
  int gm_split_only;  // group-major for split-K partials only (a single split stores plainly)
  // a product of a call that keeps no outputs for a backward (act, encode):
  // tuned on a key of its own with a minimum K split (see the launcher)
  int act;
};

inline Epi epi(float* C, int ldc, const float* bias = nullptr, int relu = 0, int accumulate = 0) {
  return Epi{C, ldc, bias, 1.0f, relu, accumulate, nullptr, 0, 1, 0, 0, 0, 0, 0, 0, 0, 0};
}

__device__ __forceinline__ size_t crow(const Epi& e, int m) {
  if (e.rq <= 0) return (size_t)m;
  const int b = m / e.rq, q = m - b * e.rq, h = q / e.rwq, w = q - h * e.rwq;
  return (size_t)b * e.rs1 + (size_t)h * e.rs2 + (size_t)w * e.rs3 + e.r0;
}

constexpr int kMaxMbEnvs = 256;
struct MapArgs {
  int F, nb, N, T;
  int env[kMaxMbEnvs];  // length-sorted (descending) env ids
  int len[kMaxMbEnvs];
};

// Benchmark aid: while g_gemm_timer is set, each GEMM launcher records
// start[n] / end[n] on its stream around the GEMM kernel itself (not the
// split-K reduction) and adds the launch's 2*M*N*K to flops, up to cap
// launches (never while the stream is being captured).
struct GemmTimer {
  hipEvent_t* start;
  hipEvent_t* end;
  int cap, n;
  double flops;
  double wbytes;  // weight operand bytes of the timed convolution products
};
extern thread_local GemmTimer* g_gemm_timer;

// GEMM tile autotuner state of one net: the fastest (tile, K split) per
// problem (operand kind, M, N, K, precision); while `tuning` is set, a problem
// not in the table is timed on its stream over every candidate before it runs
// (never inside stream capture, never for a deferred split whose partial
// tiles a consumer sums).  g_gemm_tune is set by the library entry points.
struct GemmTune {
  std::map<std::array<long long, 5>, std::pair<int, int>> best;
  int tuning = 0;
};
extern thread_local GemmTune* g_gemm_tune;

// gemm.hip (prec: 0 float32 operands, 1 bfloat16 operands)
int gemm_max_splits_for(long M, long N, long K, int prec);
constexpr int kGemmTiles = 6;  // tile shapes the autotuner's table may name
// pb: bytes of `partial` available for split-K partial tiles
// defer: leave split-K partial tiles [splits][M][N] in `partial` (no reduction
// launch); returns the split count
int gemm_conv_fwd(int prec, const ConvGeo& g, const float* x, const void* w, Epi e, size_t pb,
                  float* partial, hipStream_t s, bool defer = false);
// wt: scratch for the weights reordered to [C][KH*KW][Co] (C*KH*KW*Co elements
// of the operand type).
void gemm_conv_dgrad(int prec, const ConvGeo& g, const float* dy, const void* w, void* wt, Epi e, size_t pb,
                     float* partial, hipStream_t s);
void gemm_conv_wgrad(int prec, const ConvGeo& g, const float* x, const float* dy, Epi e, size_t pb,
                     float* partial, hipStream_t s);
// split_a: carry A as hi + lo bfloat16 parts (gradient operands of backward products)
void gemm_dense(int prec, bool ta, bool tb, const float* a, int lda, const void* b, bool b_lp, int ldb,
                int M, int N, int K, Epi e, bool split_a, size_t pb, float* partial, hipStream_t s);

// norm.hip
void launch_gn_forward(const float* y, int B, int P, int C, int G, float eps, const float* gamma,
                       const float* beta, const float* res, int relu, float* out, int out_chw,
                       float2* stats, float4* part, int S, hipStream_t s);
void launch_gn_backward(const float* dout, const float* out, int chw, const float* y, int B, int P,
                        int C, int G, const float2* stats, const float* gamma, float* dy, float* dres,
                        float* dgamma, float* dbeta, float2* bpart, float2* coef, int S, hipStream_t s);
void launch_maxpool_fwd(const float* x, int B, int H, int W, int C, float* y, uint8_t* arg,
                        hipStream_t s);
void launch_maxpool_bwd(const float* dy, const uint8_t* arg, int B, int H, int W, int C, float* dx,
                        hipStream_t s);
void launch_prep(const void* obs, int bf16, const int32_t* src, int F, int C, int Hin, int Win, int pool,
                 float* x0, hipStream_t s);
void launch_relu_grad(const float* dy, const float* y, size_t n, float* dx, hipStream_t s);
// fused GroupNorm (one workgroup per image and group); 0 = group too large
int gn_fused_npt(int P, int Cg);
// src_gm: the input (or its split-K partials) is group-major (Epi::gm_p).
// pool_out: instead of `out`, write the 3x3 / 2 (pad 1) max pool of the
// normalised H x W map (NHWC, ceil(H/2) x ceil(W/2)); needs gn_pool_fits.
// second: a GroupNorm of the same shape (its input or split-K partials, own
// affine parameters and statistics, no ReLU) whose output is the residual
// (res must then be null): a projection shortcut normalised in the same launch.
constexpr long kGnPoolLds = 64 * 1024;
struct GnSecond {
  const float* src;
  int nsplit, src_gm;
  const float *gamma, *beta;
  float2* stats;
};
bool gn_pool_fits(int P, int Cg);
void launch_gn_fused(const float* src, int nsplit, size_t zstride, float* u_out, int B, int P, int C, int G,
                     float eps, const float* gamma, const float* beta, const float* res, int relu, float* out,
                     int out_chw, float2* stats, hipStream_t s, int src_gm = 0, float* pool_out = nullptr,
                     int H = 0, int W = 0, const GnSecond* second = nullptr);
void launch_gnb_fused(const float* dout, const float* outm, int chw, const float* y, int B, int P, int C, int G,
                      const float2* stats, const float* gamma, float* dy, float* dres, float* dgamma,
                      float* dbeta, float2* bpart, hipStream_t s);

// lstm.hip
void launch_mask_state(const float* h_in, const float* c_in, const float* mask, int rows, int H,
                       float* hp, int ldhp, float* cp, hipStream_t s);
void launch_colsum(const float* in, int rows, int cols, int ld, float* out, hipStream_t s);

// lstm_step.hip: one launch per time step (see the file header)
void launch_lstm_step_fwd(int prec, const float* X, int ldx, int K, const void* W, int ldw, const float* Gin,
                          const float* bias, const float* cprev, int rows, int H, float* act, float* h_out,
                          int ldh, float* c_out, const float* mask_next, int rows_next, float* hp_next,
                          int ldhp, float* cp_next, hipStream_t s);
void launch_lstm_step_bwd(int prec, const float* dGn, const void* WT, const float* mask_n, int rows_n,
                          const float* act, const float* c, const float* cp, const float* dH, int ldd, int rows,
                          int H, float* dG, float* dcp, hipStream_t s);
// WT [H][4H] = transpose of the recurrent block W[:, din:din+H] (row stride ldw)
void launch_transpose_whh(int prec, const void* W, int ldw, int H, void* WT, hipStream_t s);

// lstm_seq.hip: one cooperative launch for all TB steps of a layer (see the
// file header).  Return 0 when launched, nonzero when the shape or the device
// does not allow it (nothing launched; the caller runs the per-step kernels).
// sync: kLstmSyncBytes of device memory owned by the call.
constexpr size_t kLstmSyncBytes = 257 * 256;
// The sticky error word of the persistent launches (uint32 at this byte
// offset of the sync area): nonzero once a barrier wait gave up and the
// launch poisoned its outputs with NaN.  Cleared by launch_lstm_clear_error.
size_t lstm_error_word_offset();
void launch_lstm_clear_error(unsigned* sync, hipStream_t s);
int launch_lstm_seq_fwd(int prec, const MapArgs& m, int TB, int H, const void* Whh, int ldw, float* G, float* HP,
                        float* CP, float* Cs, float* Ho, int ldh, const float* mskf, unsigned* sync,
                        hipStream_t s);
int launch_lstm_seq_bwd(int prec, const MapArgs& m, int TB, int H, const void* Whh, int ldw, const float* G,
                        const float* CP, const float* Cs, const float* dH, int ldd, float* dG, const float* mskf,
                        unsigned* sync, hipStream_t s);

// Both layers of a 2-layer LSTM in one cooperative launch per direction,
// pipelined one step apart (T + 1 barriers).  Forward: G0 holds x W_ih0^T + b0
// on entry; layer 1's input projection (W1 = [W_ih1 | W_hh1], [4H][2H]) and
// bias b1 are applied in-kernel; HP/CP rows of step 0 of both layers are set
// by the caller.  Backward: dHtop is the gradient at layer 1's output; writes
// dG1 and dG0 (layer 0's input gradient dG1 W_ih1 is formed in-kernel).
// Return 0 when launched, nonzero when not (nothing launched).
int launch_lstm_seq2_fwd(int prec, const MapArgs& m, int TB, int H, const void* Whh0, int ldw0, const void* W1,
                         const float* b1, float* G0, float* HP0, float* CP0, float* Cs0, float* Ho0, float* G1,
                         float* HP1, float* CP1, float* Cs1, float* Ho1, const float* mskf, unsigned* sync,
                         hipStream_t s);
int launch_lstm_seq2_bwd(int prec, const MapArgs& m, int TB, int H, const void* Whh0, int ldw0, const void* W1,
                         const float* G0, const float* CP0, const float* Cs0, const float* G1, const float* CP1,
                         const float* Cs1, const float* dHtop, float* dG0, float* dG1, const float* mskf,
                         unsigned* sync, hipStream_t s);

// lstm_act.hip: the act step's goal / embedding inputs and masked state
// (one launch), then one launch per LSTM layer (see the file header)
void launch_act_core_prep(const float* goal, const int32_t* prev_a, const float* mask, int B, int polar,
                          int goal_dim, const float* gw, const float* gb, int E, const float* emb, float* Z, int ldz,
                          int zoff, const float* h_in, const float* c_in, int L, int SR, int H, float* hm, float* cm,
                          hipStream_t s);
bool act_layer_supported(int din, int H, int B);
// SE-ResNeXt blocks (seresnext.hip): grouped 3x3 convolution (G groups,
// weights [Co][3][3][C/G]) forward, data gradient (accumulate: add into dx)
// and weight gradient (partials of at most part_bytes, then summed in order
// into dw); squeeze-excite gate forward (z, a1, gate kept for the backward;
// zpart: [kSeMaxSlices][F][C] scratch) and backward (dres: the shortcut's
// gradient, dy: the branch's; dspart: the same scratch).
constexpr int kSeMaxSlices = 16;   // pixel slices of a squeeze reduction (partial sums [S][F][C])
bool gconv_supported(const ConvGeo& g, int G);
bool gconv_fits(const ConvGeo& g);   // element counts within 31-bit indices
void launch_gconv_fwd(int prec, const ConvGeo& g, int G, const float* x, const void* w, float* y, hipStream_t s);
void launch_gconv_dgrad(int prec, const ConvGeo& g, int G, const float* dy, const void* w, float* dx,
                        int accumulate, hipStream_t s);
void launch_gconv_wgrad(int prec, const ConvGeo& g, int G, const float* x, const float* dy, float* dw,
                        float* part, size_t part_bytes, hipStream_t s);
void launch_se_forward(const float* y, const float* res, int F, int HW, int C, int R, const float* w1,
                       const float* b1, const float* w2, const float* b2, float* zpart, float* z, float* a1,
                       float* gate, float* out, hipStream_t s);
void launch_se_backward(const float* dout, const float* out, const float* y, const float* z, const float* a1,
                        const float* gate, int F, int HW, int C, int R, const float* w1, const float* w2,
                        float* dres, float* dspart, float* da2, float* da1, float* dz, float* gw1, float* gb1,
                        float* gw2, float* gb2, float* dy, hipStream_t s);

void launch_lstm_act_layer(int prec, const float* X, int ldx, int din, const float* HM, const float* CM,
                           const void* W, int ldw, const float* bias, int B, int H, float* h_out, float* c_out,
                           const int32_t* active, hipStream_t s);

// head.hip
void launch_act_head(const float* htop, int rows, int H, int A, const float* W, const float* b,
                     const float* u, int32_t* action, float* logp, float* value, float* logits,
                     const int32_t* active, hipStream_t s);
void launch_loss_head(const float* htop, int F, int H, int A, const float* W, const float* b,
                      const int32_t* src, const int32_t* actions, const float* logp_old, const float* adv,
                      const float* ret, const float* wf, float clip, float vcoef, float ecoef,
                      int norm_adv, const double* adv_stats, const float* loss_scale, float* fstat,
                      float* dout, float* dh, float* stats, hipStream_t s);
void launch_loss_terms(const float* logits, const float* values, int F, int A, const int32_t* src,
                       const int32_t* actions, const float* logp_old, const float* adv, const float* ret,
                       const float* wf, float clip, float vcoef, float ecoef, int norm_adv,
                       const double* adv_stats, const float* loss_scale, float* fstat, float* dlogits,
                       float* dvalues, float* stats, float* loss_out, hipStream_t s);
void launch_embed_fwd(const float* goal, const int32_t* prev_a, const float* mask, const int32_t* src,
                      int F, int polar, int goal_dim, const float* gw, const float* gb, int E,
                      const float* emb, float* Z, int ldz, int zoff, hipStream_t s);
void launch_embed_bwd(const float* goal, const int32_t* prev_a, const float* mask, const int32_t* src,
                      int F, int polar, int goal_dim, int E, int A1, const float* dZ, int ldz, int zoff,
                      float* dgw, float* dgb, float* demb, hipStream_t s);
void launch_relu_grad2d(const float* dy, int ldd, const float* y, int ldy, int rows, int cols, float* dx,
                        int ldx, hipStream_t s);
void launch_frame_map(const MapArgs& m, const float* mask, int32_t* src, float* w, float* msk,
                      int32_t* env_row, hipStream_t s);
void launch_gather_state(const float* srcs, int L, int N, int nb, int H, const int32_t* env_row,
                         float* dst, hipStream_t s);
void launch_copy2d(const float* s_, int lds, int rows, int cols, float* d, int ldd, hipStream_t s,
                   const int32_t* active = nullptr);
void launch_goal_dgrad(const float* dZ, int ldz, int zoff, int F, int goal_dim, const float* gw, float* dgoal,
                       hipStream_t s);
void launch_planner_goal(const float* raw, int ldr, const int32_t* dst, int F, float* goal, hipStream_t s);
void launch_planner_goal_bwd(const float* raw, int ldr, const float* dgoal, int F, float* draw, hipStream_t s);
void launch_head_fwd(const float* htop, int F, int H, int A, const float* W, const float* b, float* logits,
                     float* values, hipStream_t s);
void launch_head_bwd(const float* dlogits, const float* dvalues, int F, int H, int A, const float* W, float* dout,
                     float* dh, hipStream_t s);
void launch_copy_i32(const int32_t* src, int n, int32_t* dst, hipStream_t s);

// gae_adam.hip
void launch_gae(const float* rew, const float* val, const uint8_t* done, const int32_t* len, int T, int N,
                float gamma, float lambda, float* adv, float* ret, double* stats, hipStream_t s);
size_t adam_ws_bytes();
void launch_adam(float* th, const float* g, float* m, float* v, bf16_t* lp, size_t P, float lr, float b1,
                 float b2, float eps, int growth, ppo_scaler* sc, void* ws, hipStream_t s);
void launch_cast_bf16(const float* src, bf16_t* dst, size_t n, hipStream_t s);
