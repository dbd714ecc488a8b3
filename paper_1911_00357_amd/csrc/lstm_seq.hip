// Persistent LSTM recurrence over a packed minibatch: one cooperative launch
// per layer and direction runs every time step (Sec. 3: the recurrent core
// over a rollout of T steps; its backward is truncated BPTT over the same T).
// With two layers a single launch per direction runs both, pipelined a step
// apart (the lstm_seq2 kernels below).
//
// Work split: block b owns hidden units [b U, b U + U) of the layer for all
// steps.  Its slice of W_hh (the 4U gate rows for the forward, the U columns
// for the backward) is loaded into registers once; the cell (forward) or cell
// gradient carry (backward) of its units stays in LDS across steps.  Each
// step reads the previous step's full recurrent vector (h for the forward,
// dG for the backward) that every block wrote, so the blocks meet at a
// device-wide barrier between steps.
//
// Exchange without cache maintenance: the rows that other blocks read within
// the launch are stored as relaxed agent-scope atomics and read with 16-byte
// buffer loads carrying the same device-scope cache policy, so they are
// served where the chip's L2 slices are coherent and no L2 write-back or
// invalidate is needed (those cost 10-20 us per barrier at 256 blocks).  A
// block reads each exchanged row once per step into LDS (rounds of a few
// rows), and all of its gate columns take their operands from there.  Each
// wavefront waits for its stores to be acknowledged before the block
// barrier; thread 0 then publishes the step number in the block's own flag
// line, and every block polls all flags (one lane per flag).  The waits are
// bounded: a block that polls longer than kSpinLimit rounds stops waiting,
// sets the error word and writes NaN into its remaining outputs, so the
// kernel always ends and the failure shows as a non-finite loss or gradient.
//
// Packed rows: envs are ordered longest first, so step t covers rows
// [off[t], off[t] + act[t]) with act[t] = #{j : len_j > t} and
// off[t] = sum_j min(len_j, t); row r of step t is the minibatch's env r.
#include "common.h"
#include "kernels.h"

namespace {

constexpr int kSpinLimit = 1 << 21;  // polls of about 1 us each
constexpr int kDeviceScope = 16;     // buffer-load cache policy bit for device (agent) scope coherence
// exchanged rows staged per round (32 KB of forward rows, 32 KB of backward
// rows for one layer; 48 / 64 KB for two layers): 16 / 4 / 8 / 4 rows at H = 512
constexpr int rows_f(int H) { return 8192 / H; }   // forward, one layer
constexpr int rows_b(int H) { return 2048 / H; }   // backward, one layer (rows of 4H)
constexpr int rows_f2(int H) { return 4096 / H; }  // forward, two layers (three row sets)
constexpr int rows_b2(int H) { return 2048 / H; }  // backward, two layers (two row sets of 4H)

struct SeqArgs {
  const void* W;  // layer weights [4H][ldw]; W_hh at column offset 0 of this pointer
  int ldw;
  int H, TB, nb;
  float* G;         // [F][4H] forward: x W_ih^T + b in, gate activations out; backward: activations in
  float* HP;        // [F][H] m_t h_{t-1}
  float* CP;        // [F][H] m_t c_{t-1}
  float* Cs;        // [F][H] c_t
  float* Ho;        // [F][ldh] h_t (forward)
  int ldh;
  const float* dH;  // [F][ldd] gradient at h_t from above (backward)
  int ldd;
  float* dG;        // [F][4H] gate pre-activation gradients (backward)
  const float* mskf;  // [F] m_t per packed row
  unsigned* sync;     // [blocks] flag words at a 64-word stride (zeroed at launch); error word at kErrWord
  int len[kMaxMbEnvs];
};

DEV float bf_round(float x) { return bf2f(f2bf(x)); }

DEV void xstore(float* p, float v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

typedef __amdgpu_buffer_rsrc_t rsrc_t;
// Buffer descriptor over an exchanged array (offsets below 2^31 bytes, checked by the host).
DEV rsrc_t xrsrc(const float* p) { return __builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, 0x7fffffff, 0x00020000); }
DEV v4f xload4(rsrc_t r, uint32_t elem) {
  return __builtin_bit_cast(v4f, __builtin_amdgcn_raw_buffer_load_b128(r, elem * 4u, 0, kDeviceScope));
}

// Copies NA row sets of exchanged data into LDS: set i is n4[i] float4s from
// element e0[i] of src[i] to dst[i] (rounded to bfloat16 when bf).  Every
// load is issued before the first LDS store; NL bounds the float4s a thread
// moves per set.
template <int NL, int NA>
DEV void stage(const rsrc_t (&src)[NA], const uint32_t (&e0)[NA], const int (&n4)[NA], float* const (&dst)[NA],
               bool bf) {
  v4f v[NA][NL];
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int j = 0; j < NL; ++j) {
      const int i = threadIdx.x + 256 * j;
      if (i < n4[a]) v[a][j] = xload4(src[a], e0[a] + 4u * i);
    }
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int j = 0; j < NL; ++j) {
      const int i = threadIdx.x + 256 * j;
      if (i < n4[a]) {
        v4f x = v[a][j];
        if (bf) x = v4f{bf_round(x.x), bf_round(x.y), bf_round(x.z), bf_round(x.w)};
        *(v4f*)(dst[a] + 4 * i) = x;
      }
    }
}

// float4s per thread for `rows` rows of n floats
constexpr int stage_nl(int rows, int n) { return (rows * n / 4 + 255) / 256; }

// dot of the LDS row segment of lane s (KPT/4 float4s at stride 4 T) with w
template <int KPT, int T>
DEV float ldot(const float* row, int s, const float (&w)[KPT]) {
  const float* p = row + 4 * s;
  float acc = 0.f;
#pragma unroll
  for (int i = 0; i < KPT / 4; ++i) {
    const v4f v = *(const v4f*)(p + 4 * T * i);
    acc = fmaf(v.x, w[4 * i + 0], acc);
    acc = fmaf(v.y, w[4 * i + 1], acc);
    acc = fmaf(v.z, w[4 * i + 2], acc);
    acc = fmaf(v.w, w[4 * i + 3], acc);
  }
  return acc;
}

constexpr int kFlagStride = 64;  // words: one 256-byte line per block
// The error word sits on the line after the largest grid's flags (at most 256
// blocks, pick_units); launches clear only their flags, so a failure stays
// visible until the next learner call clears it (launch_lstm_clear_error).
constexpr int kErrWord = kFlagStride * 256;

// Barrier `gen` (1, 2, ...) of the launch; `broken` is uniform in the block.
DEV void grid_sync(unsigned* flags, unsigned gen, int& broken) {
  __builtin_amdgcn_s_waitcnt(0);  // this wavefront's exchange stores are acknowledged
  __syncthreads();
  if (threadIdx.x == 0)
    __hip_atomic_store(flags + kFlagStride * blockIdx.x, gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (broken) return;
  for (int spins = 0;; ++spins) {
    unsigned v = gen;
    if (threadIdx.x < gridDim.x)
      v = __hip_atomic_load(flags + kFlagStride * threadIdx.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (__syncthreads_and(v >= gen)) return;
    if (spins > kSpinLimit) {
      broken = 1;
      if (threadIdx.x == 0)
        __hip_atomic_store(flags + kErrWord, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

// off[t] for t in [0, TB] into LDS.
DEV void packed_offsets(const int* len, int nb, int TB, int* off) {
  for (int t = threadIdx.x; t <= TB; t += blockDim.x) {
    int s = 0;
    for (int j = 0; j < nb; ++j) s += min(len[j], t);
    off[t] = s;
  }
}

template <typename TW>
DEV float wload(const TW* p) {
  return ldf(p);
}

// Forward.  Thread layout for the products: column c = q U + u (gate q of
// unit u) takes TPC = 64/U consecutive lanes; lane s of the column holds
// W_hh[q H + j][k] for k = 4 s + 4 TPC i + e (i < KPT/4, e < 4); H = TPC KPT.
template <typename TW, int U, int KPT>
__global__ void __launch_bounds__(256) lstm_seq_fwd_kernel(SeqArgs a) {
  extern __shared__ __align__(16) float lds[];
  constexpr int TPC = 64 / U;
  constexpr int H = TPC * KPT;
  constexpr bool BF = sizeof(TW) == 2;
  constexpr int kRowsF = rows_f(H);
  int* off = (int*)lds;                      // [TB + 1]
  float* gates = lds + ((a.TB + 4) & ~3);    // [nb][4U]
  float* cst = gates + kMaxMbEnvs * 4 * U;   // [nb][U] masked c_{t-1}
  float* stg = cst + kMaxMbEnvs * U;         // [kRowsF][H] staged m_t h_{t-1} rows
  int broken = 0;
  const int j0 = blockIdx.x * U;
  const int col = threadIdx.x / TPC, s = threadIdx.x % TPC;
  const int q = col / U, uc = col % U;
  const TW* Wt = (const TW*)a.W;
  float w[KPT];
  {
    const TW* wr = Wt + (size_t)(q * H + j0 + uc) * a.ldw;
#pragma unroll
    for (int i = 0; i < KPT / 4; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) w[4 * i + e] = wload(wr + 4 * s + 4 * TPC * i + e);
  }
  const rsrc_t rHP = xrsrc(a.HP);
  packed_offsets(a.len, a.nb, a.TB, off);
  // pointwise item of this thread: row pr, unit pu (rows x U <= 256 checked by the host)
  const int pr = threadIdx.x / U, pu = threadIdx.x % U, pj = j0 + pu;
  __syncthreads();
  if (pr < off[1]) cst[pr * U + pu] = a.CP[(size_t)pr * H + pj];  // step 0: rows [0, act[0])
  __syncthreads();
  for (int t = 0; t < a.TB; ++t) {
    const int base = off[t], rows = off[t + 1] - base;
    const int nbase = off[t + 1];
    const int nrows = t + 1 < a.TB ? off[t + 2] - nbase : 0;
    const bool mine = pr < rows;
    float gin[4] = {0.f, 0.f, 0.f, 0.f}, mnext = 0.f;
    if (mine) {
      const float* g = a.G + (size_t)(base + pr) * 4 * H + pj;
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) gin[qq] = g[qq * H];
      if (pr < nrows) mnext = a.mskf[nbase + pr];
    }
    // gates_t[r][c] = sum_k HP[r][k] W[c][k]
    for (int c0 = 0; c0 < rows; c0 += kRowsF) {
      const int nr = min(kRowsF, rows - c0);
      {
        const rsrc_t src[1] = {rHP};
        const uint32_t e0[1] = {(uint32_t)(base + c0) * H};
        const int n4[1] = {nr * H / 4};
        float* const dst[1] = {stg};
        stage<stage_nl(kRowsF, H), 1>(src, e0, n4, dst, BF);
      }
      __syncthreads();
      for (int r = 0; r < nr; ++r) {
        float acc = ldot<KPT, TPC>(stg + r * H, s, w);
#pragma unroll
        for (int o = TPC / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
        if (s == 0) gates[(c0 + r) * 4 * U + col] = acc;
      }
      __syncthreads();
    }
    if (mine) {
      const float* gr = gates + pr * 4 * U + pu;
      const float ig = sigm(gr[0] + gin[0]), fg = sigm(gr[U] + gin[1]);
      const float gg = tanhf(gr[2 * U] + gin[2]), og = sigm(gr[3 * U] + gin[3]);
      const float c2 = fg * cst[pr * U + pu] + ig * gg;
      float h2 = og * tanhf(c2);
      if (broken) h2 = __builtin_nanf("");
      const size_t row = base + pr;
      float* ga = a.G + row * 4 * H + pj;
      ga[0] = ig;
      ga[H] = fg;
      ga[2 * H] = gg;
      ga[3 * H] = og;
      a.Cs[row * H + pj] = c2;
      a.Ho[row * a.ldh + pj] = h2;
      if (pr < nrows) {
        xstore(a.HP + (size_t)(nbase + pr) * H + pj, mnext * h2);
        a.CP[(size_t)(nbase + pr) * H + pj] = mnext * c2;
        cst[pr * U + pu] = mnext * c2;
      }
    }
    if (t + 1 < a.TB) grid_sync(a.sync, (unsigned)(t + 1), broken);
  }
}

// Backward.  Unit u of the block takes TPB = 256/U consecutive threads; thread
// s of the unit holds W_hh[g][j] for g = 4 s + 4 TPB i + e (i < KPT/4); 4H = TPB KPT.
template <typename TW, int U, int KPT>
__global__ void __launch_bounds__(256) lstm_seq_bwd_kernel(SeqArgs a) {
  extern __shared__ __align__(16) float lds[];
  constexpr int TPB = 256 / U;
  constexpr int WPU = TPB / 64;  // wavefronts per unit (>= 1)
  constexpr int H4 = TPB * KPT, H = H4 / 4;
  constexpr int kRowsB = rows_b(H);
  int* off = (int*)lds;                          // [TB + 1]
  float* red = lds + ((a.TB + 4) & ~3);          // [4 waves][nb]
  float* dcs = red + 4 * kMaxMbEnvs;             // [nb][U] dc carry
  float* stg = dcs + kMaxMbEnvs * U;             // [kRowsB][4H] staged dG_{t+1} rows
  int broken = 0;
  const int j0 = blockIdx.x * U;
  const int uw = threadIdx.x / TPB, s = threadIdx.x % TPB;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const TW* Wt = (const TW*)a.W;
  float w[KPT];
#pragma unroll
  for (int i = 0; i < KPT / 4; ++i)
#pragma unroll
    for (int e = 0; e < 4; ++e) w[4 * i + e] = wload(Wt + (size_t)(4 * s + 4 * TPB * i + e) * a.ldw + j0 + uw);
  const rsrc_t rdG = xrsrc(a.dG);
  packed_offsets(a.len, a.nb, a.TB, off);
  const int pr = threadIdx.x / U, pu = threadIdx.x % U, pj = j0 + pu;
  if (pr < a.nb) dcs[pr * U + pu] = 0.f;
  __syncthreads();
  for (int t = a.TB - 1; t >= 0; --t) {
    const int base = off[t], rows = off[t + 1] - base;
    const int nbase = off[t + 1];
    const int nrows = t + 1 < a.TB ? off[t + 2] - nbase : 0;
    const bool mine = pr < rows;
    float gt[4] = {0.f, 0.f, 0.f, 0.f}, cv = 0.f, cpv = 0.f, dh = 0.f, mn = 0.f;
    if (mine) {
      const size_t row = base + pr;
      const float* g = a.G + row * 4 * H + pj;
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) gt[qq] = g[qq * H];
      cv = a.Cs[row * H + pj];
      cpv = a.CP[row * H + pj];
      dh = a.dH[row * a.ldd + pj];
      if (pr < nrows) mn = a.mskf[nbase + pr];
    }
    // dHP_{t+1}[r][j] = sum_g dG_{t+1}[r][g] W_hh[g][j]
    for (int c0 = 0; c0 < nrows; c0 += kRowsB) {
      const int nr = min(kRowsB, nrows - c0);
      {
        const rsrc_t src[1] = {rdG};
        const uint32_t e0[1] = {(uint32_t)(nbase + c0) * H4};
        const int n4[1] = {nr * H};
        float* const dst[1] = {stg};
        stage<stage_nl(kRowsB, H4), 1>(src, e0, n4, dst, false);
      }
      __syncthreads();
      for (int r = 0; r < nr; ++r) {
        const float acc = wave_sum(ldot<KPT, TPB>(stg + r * H4, s, w));
        if (lane == 0) red[wave * kMaxMbEnvs + c0 + r] = acc;
      }
      __syncthreads();
    }
    if (mine) {
      float dc = 0.f;
      if (pr < nrows) {
        float sdot = 0.f;
#pragma unroll
        for (int k = 0; k < WPU; ++k) sdot += red[(pu * WPU + k) * kMaxMbEnvs + pr];
        dh += mn * sdot;
        dc = mn * dcs[pr * U + pu];
      }
      const float ig = gt[0], fg = gt[1], gg = gt[2], og = gt[3];
      const float tc = tanhf(cv);
      const float d_o = dh * tc;
      dc += dh * og * (1.f - tc * tc);
      float* d = a.dG + (size_t)(base + pr) * 4 * H + pj;
      const float nan = broken ? __builtin_nanf("") : 1.f;
      xstore(d, nan * (dc * gg * ig * (1.f - ig)));
      xstore(d + H, nan * (dc * cpv * fg * (1.f - fg)));
      xstore(d + 2 * H, nan * (dc * ig * (1.f - gg * gg)));
      xstore(d + 3 * H, nan * (d_o * og * (1.f - og)));
      dcs[pr * U + pu] = dc * fg;
    }
    if (t > 0) grid_sync(a.sync, (unsigned)(a.TB - t), broken);
  }
}

// ---------------------------------------------- two layers, pipelined
// With two layers the forward runs layer 0 at step k and layer 1 at step k-1
// in the same barrier interval (layer 1 reads layer 0's h_{k-1}, exchanged
// at the previous barrier), and the backward runs layer 1 at step t and
// layer 0 at step t+1 (layer 0's input gradient at t+1 is dG1_{t+1} W_ih1,
// the same rows layer 1's recurrence reads): T + 1 barriers for both layers
// instead of 2T, and layer 1's input projection / layer 0's input gradient
// need no separate product over all frames.
struct Seq2Args {
  const void* W0;   // layer 0 recurrent block W_hh0 (column offset applied), row stride ldw0
  int ldw0;
  const void* W1;   // layer 1 weights [4H][2H]: W_ih1 at column 0, W_hh1 at column H
  const float* b1;  // layer 1 bias [4H]
  int H, TB, nb;
  float *G0, *HP0, *CP0, *Cs0, *Ho0;  // layer 0 (G0: x W_ih0^T + b0 in, activations out)
  float *G1, *HP1, *CP1, *Cs1, *Ho1;  // layer 1 (G1: activations out)
  const float* dHtop;                 // [F][H] gradient at layer 1's output
  float *dG0, *dG1;
  const float* mskf;
  unsigned* sync;
  int len[kMaxMbEnvs];
};

template <typename TW, int U, int KPT>
__global__ void __launch_bounds__(256) lstm_seq2_fwd_kernel(Seq2Args a) {
  extern __shared__ __align__(16) float lds[];
  constexpr int TPC = 64 / U;
  constexpr int H = TPC * KPT;
  constexpr bool BF = sizeof(TW) == 2;
  constexpr int kRowsF2 = rows_f2(H);
  int* off = (int*)lds;                        // [TB + 1]
  float* g0 = lds + ((a.TB + 4) & ~3);         // [nb][4U] gates of layer 0
  float* g1 = g0 + kMaxMbEnvs * 4 * U;         // [nb][4U] gates of layer 1
  float* c0s = g1 + kMaxMbEnvs * 4 * U;        // [nb][U] masked c of layer 0
  float* c1s = c0s + kMaxMbEnvs * U;           // [nb][U] masked c of layer 1
  float* s0 = c1s + kMaxMbEnvs * U;            // [kRowsF2][H] staged m h rows of layer 0
  float* sx = s0 + kRowsF2 * H;                // [kRowsF2][H] staged h rows of layer 0 (layer 1 input)
  float* s1 = sx + kRowsF2 * H;                // [kRowsF2][H] staged m h rows of layer 1
  int broken = 0;
  const int j0 = blockIdx.x * U;
  const int col = threadIdx.x / TPC, s = threadIdx.x % TPC;
  const int q = col / U, uc = col % U;
  float w0[KPT], w1i[KPT], w1h[KPT];
  {
    const TW* r0 = (const TW*)a.W0 + (size_t)(q * H + j0 + uc) * a.ldw0;
    const TW* r1 = (const TW*)a.W1 + (size_t)(q * H + j0 + uc) * (2 * H);
#pragma unroll
    for (int i = 0; i < KPT / 4; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int k = 4 * s + 4 * TPC * i + e;
        w0[4 * i + e] = wload(r0 + k);
        w1i[4 * i + e] = wload(r1 + k);
        w1h[4 * i + e] = wload(r1 + H + k);
      }
  }
  const rsrc_t rHP0 = xrsrc(a.HP0), rHo0 = xrsrc(a.Ho0), rHP1 = xrsrc(a.HP1);
  packed_offsets(a.len, a.nb, a.TB, off);
  const int pr = threadIdx.x / U, pu = threadIdx.x % U, pj = j0 + pu;
  __syncthreads();
  if (pr < off[1]) {
    c0s[pr * U + pu] = a.CP0[(size_t)pr * H + pj];
    c1s[pr * U + pu] = a.CP1[(size_t)pr * H + pj];
  }
  __syncthreads();
  for (int k = 0; k <= a.TB; ++k) {
    const bool l0 = k < a.TB, l1 = k >= 1;
    const int t0 = k, t1 = k - 1;
    const int base0 = l0 ? off[t0] : 0, rows0 = l0 ? off[t0 + 1] - base0 : 0;
    const int nb0 = l0 ? off[t0 + 1] : 0, nrows0 = (l0 && t0 + 1 < a.TB) ? off[t0 + 2] - nb0 : 0;
    const int base1 = l1 ? off[t1] : 0, rows1 = l1 ? off[t1 + 1] - base1 : 0;
    const int nb1 = l1 ? off[t1 + 1] : 0, nrows1 = (l1 && t1 + 1 < a.TB) ? off[t1 + 2] - nb1 : 0;
    // pointwise inputs of this thread's items (layer 0 and layer 1, row pr)
    float gin[4] = {0.f, 0.f, 0.f, 0.f}, bias1[4] = {0.f, 0.f, 0.f, 0.f}, mn0 = 0.f, mn1 = 0.f;
    if (pr < rows0) {
      const float* g = a.G0 + (size_t)(base0 + pr) * 4 * H + pj;
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) gin[qq] = g[qq * H];
      if (pr < nrows0) mn0 = a.mskf[nb0 + pr];
    }
    if (pr < rows1) {
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) bias1[qq] = a.b1[qq * H + pj];
      if (pr < nrows1) mn1 = a.mskf[nb1 + pr];
    }
    // layer 0: m h_{k-1} W_hh0^T; layer 1: h0_{k-1} W_ih1^T + m h1_{k-2} W_hh1^T
    const int rmax = max(rows0, rows1);
    for (int c0 = 0; c0 < rmax; c0 += kRowsF2) {
      const int n0 = max(0, min(kRowsF2, rows0 - c0)), n1 = max(0, min(kRowsF2, rows1 - c0));
      {
        const rsrc_t src[3] = {rHP0, rHo0, rHP1};
        const uint32_t e0[3] = {(uint32_t)(base0 + c0) * H, (uint32_t)(base1 + c0) * H,
                                (uint32_t)(base1 + c0) * H};
        const int n4[3] = {n0 * H / 4, n1 * H / 4, n1 * H / 4};
        float* const dst[3] = {s0, sx, s1};
        stage<stage_nl(kRowsF2, H), 3>(src, e0, n4, dst, BF);
      }
      __syncthreads();
      for (int r = 0; r < max(n0, n1); ++r) {
        float acc0 = r < n0 ? ldot<KPT, TPC>(s0 + r * H, s, w0) : 0.f;
        float acc1 = r < n1 ? ldot<KPT, TPC>(sx + r * H, s, w1i) + ldot<KPT, TPC>(s1 + r * H, s, w1h) : 0.f;
#pragma unroll
        for (int o = TPC / 2; o > 0; o >>= 1) {
          acc0 += __shfl_xor(acc0, o, kWave);
          acc1 += __shfl_xor(acc1, o, kWave);
        }
        if (s == 0) {
          if (r < n0) g0[(c0 + r) * 4 * U + col] = acc0;
          if (r < n1) g1[(c0 + r) * 4 * U + col] = acc1;
        }
      }
      __syncthreads();
    }
    const float nan = broken ? __builtin_nanf("") : 1.f;
    if (pr < rows0) {
      const float* gr = g0 + pr * 4 * U + pu;
      const float ig = sigm(gr[0] + gin[0]), fg = sigm(gr[U] + gin[1]);
      const float gg = tanhf(gr[2 * U] + gin[2]), og = sigm(gr[3 * U] + gin[3]);
      const float c2 = fg * c0s[pr * U + pu] + ig * gg;
      const float h2 = nan * og * tanhf(c2);
      const size_t row = base0 + pr;
      float* ga = a.G0 + row * 4 * H + pj;
      ga[0] = ig;
      ga[H] = fg;
      ga[2 * H] = gg;
      ga[3 * H] = og;
      a.Cs0[row * H + pj] = c2;
      xstore(a.Ho0 + row * H + pj, h2);
      if (pr < nrows0) {
        xstore(a.HP0 + (size_t)(nb0 + pr) * H + pj, mn0 * h2);
        a.CP0[(size_t)(nb0 + pr) * H + pj] = mn0 * c2;
        c0s[pr * U + pu] = mn0 * c2;
      }
    }
    if (pr < rows1) {
      const float* gr = g1 + pr * 4 * U + pu;
      const float ig = sigm(gr[0] + bias1[0]), fg = sigm(gr[U] + bias1[1]);
      const float gg = tanhf(gr[2 * U] + bias1[2]), og = sigm(gr[3 * U] + bias1[3]);
      const float c2 = fg * c1s[pr * U + pu] + ig * gg;
      const float h2 = nan * og * tanhf(c2);
      const size_t row = base1 + pr;
      float* ga = a.G1 + row * 4 * H + pj;
      ga[0] = ig;
      ga[H] = fg;
      ga[2 * H] = gg;
      ga[3 * H] = og;
      a.Cs1[row * H + pj] = c2;
      a.Ho1[row * H + pj] = h2;
      if (pr < nrows1) {
        xstore(a.HP1 + (size_t)(nb1 + pr) * H + pj, mn1 * h2);
        a.CP1[(size_t)(nb1 + pr) * H + pj] = mn1 * c2;
        c1s[pr * U + pu] = mn1 * c2;
      }
    }
    if (k < a.TB) grid_sync(a.sync, (unsigned)(k + 1), broken);
  }
}

template <typename TW, int U, int KPT>
__global__ void __launch_bounds__(256) lstm_seq2_bwd_kernel(Seq2Args a) {
  extern __shared__ __align__(16) float lds[];
  constexpr int TPB = 256 / U;
  constexpr int WPU = TPB / 64;
  constexpr int H4 = TPB * KPT, H = H4 / 4;
  constexpr int kRowsB2 = rows_b2(H);
  int* off = (int*)lds;                        // [TB + 1]
  float* r1 = lds + ((a.TB + 4) & ~3);         // [4 waves][nb]: dG1_{t+1} W_hh1 (layer 1 carry)
  float* rx = r1 + 4 * kMaxMbEnvs;             // [4 waves][nb]: dG1_{t0} W_ih1 (layer 0 input gradient)
  float* r0 = rx + 4 * kMaxMbEnvs;             // [4 waves][nb]: dG0_{t0+1} W_hh0 (layer 0 carry)
  float* d1s = r0 + 4 * kMaxMbEnvs;            // [nb][U] dc carries
  float* d0s = d1s + kMaxMbEnvs * U;
  float* s1 = d0s + kMaxMbEnvs * U;            // [kRowsB2][4H] staged dG1 rows
  float* s0 = s1 + kRowsB2 * H4;               // [kRowsB2][4H] staged dG0 rows
  int broken = 0;
  const int j0 = blockIdx.x * U;
  const int uw = threadIdx.x / TPB, s = threadIdx.x % TPB;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float w0[KPT], w1i[KPT], w1h[KPT];
  {
    const TW* W0 = (const TW*)a.W0;
    const TW* W1 = (const TW*)a.W1;
#pragma unroll
    for (int i = 0; i < KPT / 4; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int g = 4 * s + 4 * TPB * i + e;
        w0[4 * i + e] = wload(W0 + (size_t)g * a.ldw0 + j0 + uw);
        w1i[4 * i + e] = wload(W1 + (size_t)g * 2 * H + j0 + uw);
        w1h[4 * i + e] = wload(W1 + (size_t)g * 2 * H + H + j0 + uw);
      }
  }
  const rsrc_t rdG1 = xrsrc(a.dG1), rdG0 = xrsrc(a.dG0);
  packed_offsets(a.len, a.nb, a.TB, off);
  const int pr = threadIdx.x / U, pu = threadIdx.x % U, pj = j0 + pu;
  if (pr < a.nb) {
    d1s[pr * U + pu] = 0.f;
    d0s[pr * U + pu] = 0.f;
  }
  __syncthreads();
  auto cell_bwd = [&](const float* G, const float* Cs, const float* CP, size_t row, float dh, float dc,
                      float* dG, float nan) -> float {
    const float* gp = G + row * 4 * H + pj;
    const float ig = gp[0], fg = gp[H], gg = gp[2 * H], og = gp[3 * H];
    const float tc = tanhf(Cs[row * H + pj]);
    const float d_o = dh * tc;
    dc += dh * og * (1.f - tc * tc);
    float* d = dG + row * 4 * H + pj;
    xstore(d, nan * (dc * gg * ig * (1.f - ig)));
    xstore(d + H, nan * (dc * CP[row * H + pj] * fg * (1.f - fg)));
    xstore(d + 2 * H, nan * (dc * ig * (1.f - gg * gg)));
    xstore(d + 3 * H, nan * (d_o * og * (1.f - og)));
    return dc * fg;
  };
  for (int k = 0; k <= a.TB; ++k) {
    const int t1 = a.TB - 1 - k, t0 = a.TB - k;  // layer 1 step, layer 0 step
    const bool l1 = t1 >= 0, l0 = k >= 1;
    // exchanged rows: dG1 of step t0 (= t1 + 1) and dG0 of step t0 + 1
    const int be = (t0 < a.TB) ? off[t0] : 0, re = (t0 < a.TB) ? off[t0 + 1] - be : 0;
    const int bd = (l0 && t0 + 1 < a.TB) ? off[t0 + 1] : 0;
    const int rd = (l0 && t0 + 1 < a.TB) ? off[t0 + 2] - bd : 0;
    for (int c0 = 0; c0 < re; c0 += kRowsB2) {  // rd <= re
      const int n1 = min(kRowsB2, re - c0), nd = max(0, min(kRowsB2, rd - c0));
      {
        const rsrc_t src[2] = {rdG1, rdG0};
        const uint32_t e0[2] = {(uint32_t)(be + c0) * H4, (uint32_t)(bd + c0) * H4};
        const int n4[2] = {n1 * H, nd * H};
        float* const dst[2] = {s1, s0};
        stage<stage_nl(kRowsB2, H4), 2>(src, e0, n4, dst, false);
      }
      __syncthreads();
      for (int r = 0; r < n1; ++r) {
        const float a1 = l1 ? wave_sum(ldot<KPT, TPB>(s1 + r * H4, s, w1h)) : 0.f;
        const float ax = l0 ? wave_sum(ldot<KPT, TPB>(s1 + r * H4, s, w1i)) : 0.f;
        const float a0 = r < nd ? wave_sum(ldot<KPT, TPB>(s0 + r * H4, s, w0)) : 0.f;
        if (lane == 0) {
          r1[wave * kMaxMbEnvs + c0 + r] = a1;
          rx[wave * kMaxMbEnvs + c0 + r] = ax;
          r0[wave * kMaxMbEnvs + c0 + r] = a0;
        }
      }
      __syncthreads();
    }
    const float nan = broken ? __builtin_nanf("") : 1.f;
    auto wsum = [&](const float* red, int r) {
      float v = 0.f;
#pragma unroll
      for (int q = 0; q < WPU; ++q) v += red[(pu * WPU + q) * kMaxMbEnvs + r];
      return v;
    };
    if (l1) {
      const int b1r = off[t1], n1 = off[t1 + 1] - b1r;
      if (pr < n1) {
        float dh = a.dHtop[(size_t)(b1r + pr) * H + pj], dc = 0.f;
        if (pr < re) {
          const float m = a.mskf[be + pr];
          dh += m * wsum(r1, pr);
          dc = m * d1s[pr * U + pu];
        }
        d1s[pr * U + pu] = cell_bwd(a.G1, a.Cs1, a.CP1, b1r + pr, dh, dc, a.dG1, nan);
      }
    }
    if (l0) {
      const int b0r = off[t0], n0 = off[t0 + 1] - b0r;
      if (pr < n0) {
        float dh = wsum(rx, pr), dc = 0.f;
        if (pr < rd) {
          const float m = a.mskf[bd + pr];
          dh += m * wsum(r0, pr);
          dc = m * d0s[pr * U + pu];
        }
        d0s[pr * U + pu] = cell_bwd(a.G0, a.Cs0, a.CP0, b0r + pr, dh, dc, a.dG0, nan);
      }
    }
    if (k < a.TB) grid_sync(a.sync, (unsigned)(k + 1), broken);
  }
}

__global__ void zero_sync_kernel(unsigned* p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

// Units per block: the smallest U (1, 2, 4) with H U a multiple of 256 and
// at most 256 blocks; 0 when no such U keeps KPT = H U / 64 within 64
// (H = 1024: U = 4, KPT = 64) or H outside [64, 1024].
int pick_units(int H) {
  if (H < 64 || H > 1024) return 0;
  for (int U = 1; U <= 4; U *= 2)
    if ((H * U) % 256 == 0 && H / U <= 256 && H * U / 64 <= 64) return U;
  return 0;
}

template <int U, int KPT>
const void* seq_kernel(int prec, bool bwd) {
  if (bwd)
    return prec ? (const void*)lstm_seq_bwd_kernel<bf16_t, U, KPT> : (const void*)lstm_seq_bwd_kernel<float, U, KPT>;
  return prec ? (const void*)lstm_seq_fwd_kernel<bf16_t, U, KPT> : (const void*)lstm_seq_fwd_kernel<float, U, KPT>;
}

const void* pick_kernel(int prec, bool bwd, int U, int KPT) {
#define SEQ_CASE(U_, K_) \
  if (U == U_ && KPT == K_) return seq_kernel<U_, K_>(prec, bwd);
  SEQ_CASE(1, 4) SEQ_CASE(1, 8) SEQ_CASE(1, 16) SEQ_CASE(1, 32)
  SEQ_CASE(2, 4) SEQ_CASE(2, 8) SEQ_CASE(2, 16) SEQ_CASE(2, 32)
  SEQ_CASE(4, 4) SEQ_CASE(4, 8) SEQ_CASE(4, 16) SEQ_CASE(4, 32) SEQ_CASE(4, 64)
#undef SEQ_CASE
  return nullptr;
}

int launch_seq(int prec, bool bwd, const MapArgs& m, int TB, int H, const void* W, int ldw, float* G, float* HP,
               float* CP, float* Cs, float* Ho, int ldh, const float* dH, int ldd, float* dG, const float* mskf,
               unsigned* sync, hipStream_t s) {
  const int U = pick_units(H);
  if (!U || m.nb * U > 256 || TB > 4096 || TB <= 0) return 1;
  const int KPT = H * U / 64;
  const void* k = pick_kernel(prec, bwd, U, KPT);
  if (!k) return 1;
  const size_t stg = bwd ? (size_t)rows_b(H) * 4 * H : (size_t)rows_f(H) * H;
  const size_t shmem =
      (size_t)(((TB + 4) & ~3) + (bwd ? 4 : 4 * U) * kMaxMbEnvs + kMaxMbEnvs * U + stg) * sizeof(float);
  if ((long)m.F * 4 * H * 4 >= 0x7fffffffL) return 1;  // exchange offsets are 32-bit
  const int nblk = H / U;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 1;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 256, shmem) != hipSuccess) return 1;
  if ((long)per_cu * cus < nblk) return 1;
  SeqArgs a{};
  a.W = W;
  a.ldw = ldw;
  a.H = H;
  a.TB = TB;
  a.nb = m.nb;
  a.G = G;
  a.HP = HP;
  a.CP = CP;
  a.Cs = Cs;
  a.Ho = Ho;
  a.ldh = ldh;
  a.dH = dH;
  a.ldd = ldd;
  a.dG = dG;
  a.mskf = mskf;
  a.sync = sync;
  for (int j = 0; j < m.nb; ++j) a.len[j] = m.len[j];
  const int nsync = kFlagStride * nblk;  // the flags; the error word is kept
  hipLaunchKernelGGL(zero_sync_kernel, dim3(cdiv(nsync, 256)), dim3(256), 0, s, sync, nsync);
  void* args[] = {&a};
  if (hipLaunchCooperativeKernel(k, dim3(nblk), dim3(256), args, (unsigned)shmem, s) != hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  return 0;
}

bool seq_enabled() {
  const char* e = getenv("DDPPO_LSTM_SEQ");
  return !(e && e[0] == '0');
}

bool seq2_enabled() {
  const char* e = getenv("DDPPO_LSTM_SEQ2");
  return seq_enabled() && !(e && e[0] == '0');
}

template <int U, int KPT>
const void* seq2_kernel(int prec, bool bwd) {
  if (bwd)
    return prec ? (const void*)lstm_seq2_bwd_kernel<bf16_t, U, KPT> : (const void*)lstm_seq2_bwd_kernel<float, U, KPT>;
  return prec ? (const void*)lstm_seq2_fwd_kernel<bf16_t, U, KPT> : (const void*)lstm_seq2_fwd_kernel<float, U, KPT>;
}

const void* pick_kernel2(int prec, bool bwd, int U, int KPT) {
#define SEQ2_CASE(U_, K_) \
  if (U == U_ && KPT == K_) return seq2_kernel<U_, K_>(prec, bwd);
  SEQ2_CASE(1, 4) SEQ2_CASE(1, 8) SEQ2_CASE(1, 16) SEQ2_CASE(1, 32)
  SEQ2_CASE(2, 4) SEQ2_CASE(2, 8) SEQ2_CASE(2, 16) SEQ2_CASE(2, 32)
  SEQ2_CASE(4, 4) SEQ2_CASE(4, 8) SEQ2_CASE(4, 16) SEQ2_CASE(4, 32) SEQ2_CASE(4, 64)
#undef SEQ2_CASE
  return nullptr;
}

int launch_seq2(int prec, bool bwd, const MapArgs& m, int TB, Seq2Args& a, hipStream_t s) {
  const int H = a.H;
  const int U = pick_units(H);
  if (!seq2_enabled() || !U || m.nb * U > 256 || TB > 4096 || TB <= 0) return 1;
  const int KPT = H * U / 64;
  const void* k = pick_kernel2(prec, bwd, U, KPT);
  if (!k) return 1;
  const size_t nf = bwd ? (size_t)3 * 4 * kMaxMbEnvs + 2 * kMaxMbEnvs * U + 2 * rows_b2(H) * 4 * H
                        : (size_t)2 * kMaxMbEnvs * 4 * U + 2 * kMaxMbEnvs * U + 3 * rows_f2(H) * H;
  const size_t shmem = (((TB + 4) & ~3) + nf) * sizeof(float);
  if ((long)m.F * 4 * H * 4 >= 0x7fffffffL) return 1;  // exchange offsets are 32-bit
  const int nblk = H / U;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 1;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 256, shmem) != hipSuccess) return 1;
  if ((long)per_cu * cus < nblk) return 1;
  a.TB = TB;
  a.nb = m.nb;
  for (int j = 0; j < m.nb; ++j) a.len[j] = m.len[j];
  const int nsync = kFlagStride * nblk;  // the flags; the error word is kept
  hipLaunchKernelGGL(zero_sync_kernel, dim3(cdiv(nsync, 256)), dim3(256), 0, s, a.sync, nsync);
  void* args[] = {&a};
  if (hipLaunchCooperativeKernel(k, dim3(nblk), dim3(256), args, (unsigned)shmem, s) != hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  return 0;
}

}  // namespace

void launch_lstm_clear_error(unsigned* sync, hipStream_t s) {
  hipLaunchKernelGGL(zero_sync_kernel, dim3(1), dim3(64), 0, s, sync + kErrWord, 1);
}

size_t lstm_error_word_offset() { return (size_t)kErrWord * sizeof(unsigned); }

int launch_lstm_seq_fwd(int prec, const MapArgs& m, int TB, int H, const void* Whh, int ldw, float* G, float* HP,
                        float* CP, float* Cs, float* Ho, int ldh, const float* mskf, unsigned* sync,
                        hipStream_t s) {
  if (!seq_enabled()) return 1;
  return launch_seq(prec, false, m, TB, H, Whh, ldw, G, HP, CP, Cs, Ho, ldh, nullptr, 0, nullptr, mskf, sync, s);
}

int launch_lstm_seq_bwd(int prec, const MapArgs& m, int TB, int H, const void* Whh, int ldw, const float* G,
                        const float* CP, const float* Cs, const float* dH, int ldd, float* dG, const float* mskf,
                        unsigned* sync, hipStream_t s) {
  if (!seq_enabled()) return 1;
  return launch_seq(prec, true, m, TB, H, Whh, ldw, const_cast<float*>(G), nullptr, const_cast<float*>(CP),
                    const_cast<float*>(Cs), nullptr, 0, dH, ldd, dG, mskf, sync, s);
}

int launch_lstm_seq2_fwd(int prec, const MapArgs& m, int TB, int H, const void* Whh0, int ldw0, const void* W1,
                         const float* b1, float* G0, float* HP0, float* CP0, float* Cs0, float* Ho0, float* G1,
                         float* HP1, float* CP1, float* Cs1, float* Ho1, const float* mskf, unsigned* sync,
                         hipStream_t s) {
  Seq2Args a{};
  a.W0 = Whh0;
  a.ldw0 = ldw0;
  a.W1 = W1;
  a.b1 = b1;
  a.H = H;
  a.G0 = G0;
  a.HP0 = HP0;
  a.CP0 = CP0;
  a.Cs0 = Cs0;
  a.Ho0 = Ho0;
  a.G1 = G1;
  a.HP1 = HP1;
  a.CP1 = CP1;
  a.Cs1 = Cs1;
  a.Ho1 = Ho1;
  a.mskf = mskf;
  a.sync = sync;
  return launch_seq2(prec, false, m, TB, a, s);
}

int launch_lstm_seq2_bwd(int prec, const MapArgs& m, int TB, int H, const void* Whh0, int ldw0, const void* W1,
                         const float* G0, const float* CP0, const float* Cs0, const float* G1, const float* CP1,
                         const float* Cs1, const float* dHtop, float* dG0, float* dG1, const float* mskf,
                         unsigned* sync, hipStream_t s) {
  Seq2Args a{};
  a.W0 = Whh0;
  a.ldw0 = ldw0;
  a.W1 = W1;
  a.H = H;
  a.G0 = const_cast<float*>(G0);
  a.CP0 = const_cast<float*>(CP0);
  a.Cs0 = const_cast<float*>(Cs0);
  a.G1 = const_cast<float*>(G1);
  a.CP1 = const_cast<float*>(CP1);
  a.Cs1 = const_cast<float*>(Cs1);
  a.dHtop = dHtop;
  a.dG0 = dG0;
  a.dG1 = dG1;
  a.mskf = mskf;
  a.sync = sync;
  return launch_seq2(prec, true, m, TB, a, s);
}
