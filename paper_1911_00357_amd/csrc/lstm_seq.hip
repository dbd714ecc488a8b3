// Persistent LSTM recurrence over a packed minibatch: one cooperative launch
// per layer and direction runs every time step (Sec. 3: the recurrent core
// over a rollout of T steps; its backward is truncated BPTT over the same T).
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
// the launch are stored and loaded as relaxed agent-scope atomics, which go
// to the level where the chip's L2 slices are coherent, so no L2 write-back
// or invalidate is needed (those cost 10-20 us per barrier at 256 blocks).
// Each wavefront waits for its stores to be acknowledged before the block
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
  unsigned* sync;     // [blocks] flag words at a 64-word stride, then the error word; zero at launch
  int len[kMaxMbEnvs];
};

DEV float bf_round(float x) { return bf2f(f2bf(x)); }

DEV float xload(const float* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
DEV void xstore(float* p, float v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

constexpr int kFlagStride = 64;  // words: one 256-byte line per block

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
        __hip_atomic_store(flags + kFlagStride * gridDim.x, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

// off[t] for t in [0, TB] into LDS.
DEV void packed_offsets(const SeqArgs& a, int* off) {
  for (int t = threadIdx.x; t <= a.TB; t += blockDim.x) {
    int s = 0;
    for (int j = 0; j < a.nb; ++j) s += min(a.len[j], t);
    off[t] = s;
  }
}

template <typename TW>
DEV float wload(const TW* p) {
  return ldf(p);
}

// Forward.  Thread layout for the products: column c = q U + u (gate q of
// unit u) takes TPC = 64/U consecutive lanes; lane s of the column holds
// W_hh[q H + j][k] for k = 4 s + 4 TPC i + e (i < KPT/4, e < 4).
template <typename TW, int U, int KPT>
__global__ void __launch_bounds__(256) lstm_seq_fwd_kernel(SeqArgs a) {
  extern __shared__ float lds[];
  constexpr int TPC = 64 / U;
  const int H = a.H;
  int* off = (int*)lds;                      // [TB + 1]
  float* gates = lds + ((a.TB + 4) & ~3);    // [nb][4U]
  float* cst = gates + kMaxMbEnvs * 4 * U;   // [nb][U] masked c_{t-1}
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
  packed_offsets(a, off);
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
    for (int r = 0; r < rows; ++r) {
      const float* hp = a.HP + (size_t)(base + r) * H + 4 * s;
      float acc = 0.f;
#pragma unroll
      for (int i = 0; i < KPT / 4; ++i) {
        const float* hq = hp + 4 * TPC * i;
        const float4 v = make_float4(xload(hq), xload(hq + 1), xload(hq + 2), xload(hq + 3));
        if constexpr (sizeof(TW) == 2) {
          acc = fmaf(bf_round(v.x), w[4 * i + 0], acc);
          acc = fmaf(bf_round(v.y), w[4 * i + 1], acc);
          acc = fmaf(bf_round(v.z), w[4 * i + 2], acc);
          acc = fmaf(bf_round(v.w), w[4 * i + 3], acc);
        } else {
          acc = fmaf(v.x, w[4 * i + 0], acc);
          acc = fmaf(v.y, w[4 * i + 1], acc);
          acc = fmaf(v.z, w[4 * i + 2], acc);
          acc = fmaf(v.w, w[4 * i + 3], acc);
        }
      }
#pragma unroll
      for (int o = TPC / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
      if (s == 0) gates[r * 4 * U + col] = acc;
    }
    __syncthreads();
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
// s of the unit holds W_hh[g][j] for g = 4 s + 4 TPB i + e (i < KPT/4).
template <typename TW, int U, int KPT>
__global__ void __launch_bounds__(256) lstm_seq_bwd_kernel(SeqArgs a) {
  extern __shared__ float lds[];
  constexpr int TPB = 256 / U;
  constexpr int WPU = TPB / 64;  // wavefronts per unit (>= 1)
  const int H = a.H;
  int* off = (int*)lds;                          // [TB + 1]
  float* red = lds + ((a.TB + 4) & ~3);          // [4 waves][nb]
  float* dcs = red + 4 * kMaxMbEnvs;             // [nb][U] dc carry
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
  packed_offsets(a, off);
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
    for (int r = 0; r < nrows; ++r) {
      const float* dg = a.dG + (size_t)(nbase + r) * 4 * H + 4 * s;
      float acc = 0.f;
#pragma unroll
      for (int i = 0; i < KPT / 4; ++i) {
        const float* dq = dg + 4 * TPB * i;
        const float4 v = make_float4(xload(dq), xload(dq + 1), xload(dq + 2), xload(dq + 3));
        acc = fmaf(v.x, w[4 * i + 0], acc);
        acc = fmaf(v.y, w[4 * i + 1], acc);
        acc = fmaf(v.z, w[4 * i + 2], acc);
        acc = fmaf(v.w, w[4 * i + 3], acc);
      }
      acc = wave_sum(acc);
      if (lane == 0) red[wave * kMaxMbEnvs + r] = acc;
    }
    __syncthreads();
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

__global__ void zero_sync_kernel(unsigned* p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

// Units per block: the smallest U (1, 2, 4) with H U a multiple of 256 and
// at most 256 blocks; 0 when no such U keeps KPT = H U / 64 within 32.
int pick_units(int H) {
  for (int U = 1; U <= 4; U *= 2)
    if ((H * U) % 256 == 0 && H / U <= 256 && H * U / 64 <= 32) return U;
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
  SEQ_CASE(4, 4) SEQ_CASE(4, 8) SEQ_CASE(4, 16) SEQ_CASE(4, 32)
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
  const size_t shmem = (size_t)(((TB + 4) & ~3) + kMaxMbEnvs * 4 * U + kMaxMbEnvs * U) * sizeof(float);
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
  const int nsync = kFlagStride * (nblk + 1);
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

}  // namespace

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
