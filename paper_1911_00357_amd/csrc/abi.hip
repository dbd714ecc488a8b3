// C ABI of the DD-PPO worker hot path: network plan, workspace layout and the
// host-side sequencing of the kernels for ppo_act, ppo_gae, ppo_loss_backward
// and ppo_adam_step.  Host code only launches; every step runs on the GPU.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "kernels.h"

namespace {

thread_local std::string g_err;

ppo_status fail(ppo_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

constexpr float kGnEps = 1e-5f;
constexpr size_t kSplitKBytes = 64u << 20;  // split-K partial tiles

struct Tensor {
  std::string name;
  size_t off, count;
};

// One convolution (no bias) followed by GroupNorm.
struct Unit {
  std::string name;           // convolution tensor name
  int relu;                   // 1: the stored output is post-ReLU
  size_t w, g, b;             // parameter offsets
  int Cin, Cout, K, stride, pad;
  int Hin, Win, Hout, Wout;
  int S;                      // GroupNorm pixel chunks
  int groups;                 // convolution groups (1: dense, implicit GEMM)
  size_t u, a, st;            // workspace offsets: conv out, norm out, stats (per frame sizes below)
};

struct Block {
  int c1, c2, c3, ds;         // unit indices (ds = -1: identity shortcut)
  int R;                      // squeeze-excite hidden width (0: no gate)
  size_t se1w, se1b, se2w, se2b;  // gate parameters: W1 [R][C], b1 [R], W2 [C][R], b2 [C]
};

}  // namespace

struct ppo_net {
  ppo_net_desc d;
  int prec;                   // 0 float32 operands, 1 bfloat16
  std::vector<Tensor> tensors;
  size_t P = 0;
  std::vector<Unit> units;
  std::vector<Block> blocks;
  int stem = -1;              // resnet stem unit
  int compress = -1;          // resnet compress unit (or last tiny unit)
  int h0, w0;                 // trunk input spatial size
  int pool_h, pool_w;         // resnet max pool output size
  int feat_c, feat_hw, flat;
  int din0;                   // LSTM layer-0 input width
  int emb_rows = 0;           // previous-action embedding rows (actions + start token)
  size_t fc_w, fc_b, goal_w, goal_b, emb, head_w, head_b;
  std::vector<size_t> lstm_w, lstm_b;
  // per-frame float counts used by the workspace planner
  size_t max_unit = 0;        // largest conv output per frame
  size_t gn_part = 0;         // largest S*C per frame
  int max_G = 0;
  int se_C = 0, se_R = 0;     // widest squeeze-excite gate (channels, hidden)
  // GEMM launch timer (benchmark aid, ppo_gemm_timer_arm)
  mutable int timer_unit = -1, timer_op = -1;
  mutable std::vector<hipEvent_t> timer_ev;
  mutable GemmTimer timer{};
  mutable GemmTune tune;      // tile / K-split choices (ppo_autotune)
  // ppo_collect's captured act loops, keyed on the call's arguments, oldest first
  std::unordered_map<std::string, hipGraphExec_t> graphs;
  std::deque<std::string> graph_order;
  hipStream_t cap_stream = nullptr;  // private capture stream (default priority)
  int cap_device = -1;
};

// Makes the net's tile table visible to the GEMM launchers for one call.
struct TuneScope {
  explicit TuneScope(const ppo_net* n) { g_gemm_tune = n ? &n->tune : nullptr; }
  ~TuneScope() { g_gemm_tune = nullptr; }
};

namespace {

size_t add_tensor(ppo_net* n, const std::string& name, size_t count) {
  n->tensors.push_back({name, n->P, count});
  n->P += count;
  return n->tensors.back().off;
}

int add_unit(ppo_net* n, const std::string& name, int cin, int cout, int k, int stride, int pad, int hin,
             int win, int groups = 1) {
  Unit u{};
  u.name = name;
  u.relu = 1;
  u.groups = groups;
  u.w = add_tensor(n, name, (size_t)cout * k * k * (cin / groups));
  u.g = add_tensor(n, name + ".gn.g", cout);
  u.b = add_tensor(n, name + ".gn.b", cout);
  u.Cin = cin;
  u.Cout = cout;
  u.K = k;
  u.stride = stride;
  u.pad = pad;
  u.Hin = hin;
  u.Win = win;
  u.Hout = (hin + 2 * pad - k) / stride + 1;
  u.Wout = (win + 2 * pad - k) / stride + 1;
  const int P = u.Hout * u.Wout;
  u.S = std::max(1, std::min(32, P / 64));
  n->units.push_back(u);
  n->max_unit = std::max(n->max_unit, (size_t)P * cout);
  n->gn_part = std::max(n->gn_part, (size_t)u.S * cout);
  return (int)n->units.size() - 1;
}

ConvGeo geo(const Unit& u, int F);

ppo_status build(ppo_net* n) {
  const ppo_net_desc& d = n->d;
  if (d.in_ch <= 0 || d.in_hw <= 0 || d.gn_groups <= 0 || d.hidden <= 0 || d.num_actions <= 1 ||
      d.num_actions + 1 > 8 || d.lstm_layers < 1 || d.lstm_layers > 4 || d.vis_hidden <= 0)
    return fail(PPO_ESHAPE, "invalid network sizes");
  if (d.dtype != PPO_F32 && d.dtype != PPO_BF16) return fail(PPO_EINVAL, "dtype must be F32 or BF16");
  n->prec = d.dtype == PPO_BF16 ? 1 : 0;
  int hw = d.avgpool ? d.in_hw / 2 : d.in_hw;
  if (d.avgpool && (d.in_hw & 1)) return fail(PPO_ESHAPE, "in_hw must be even with avgpool");
  n->h0 = n->w0 = hw;
  const int G = d.gn_groups;
  n->max_G = G;
  if (d.trunk == PPO_TRUNK_NONE) {
    // features in: the visual FC reads in_ch-wide float32 vectors
    if (d.in_hw != 1 || d.avgpool) return fail(PPO_ESHAPE, "a features-in net has in_hw 1 and no pooling");
    n->h0 = n->w0 = 1;
    n->feat_c = d.in_ch;
    n->feat_hw = 1;
  } else if (d.trunk == PPO_TRUNK_TINY) {
    const int c1 = d.tiny_ch[0], c2 = d.tiny_ch[1];
    if (c1 % G || c2 % G || c1 % 4 || c2 % 4) return fail(PPO_ESHAPE, "tiny widths must divide by groups and 4");
    int u1 = add_unit(n, "enc.conv1", d.in_ch, c1, 3, 2, 1, hw, hw);
    const Unit& U1 = n->units[u1];
    int u2 = add_unit(n, "enc.conv2", c1, c2, 3, 2, 1, U1.Hout, U1.Wout);
    n->compress = u2;
    n->feat_c = c2;
    n->feat_hw = n->units[u2].Hout;
    if (n->units[u2].Hout != n->units[u2].Wout) return fail(PPO_ESHAPE, "non-square map");
  } else if (d.trunk == PPO_TRUNK_RESNET || d.trunk == PPO_TRUNK_SERESNEXT) {
    const int w0 = d.base_width;
    const bool se = d.trunk == PPO_TRUNK_SERESNEXT;
    if (hw % 32) return fail(PPO_ESHAPE, "resnet trunk needs a multiple of 32 after pooling");
    if (w0 % G || w0 % 4 || d.compress_ch % G || d.compress_ch % 4)
      return fail(PPO_ESHAPE, "widths must divide by the group count and 4");
    if (se && (d.cardinality <= 0 || d.se_reduction <= 0))
      return fail(PPO_ESHAPE, "seresnext needs a positive cardinality and squeeze-excite reduction");
    n->stem = add_unit(n, "enc.stem", d.in_ch, w0, 7, 2, 3, hw, hw);
    const Unit& S = n->units[n->stem];
    n->pool_h = (S.Hout - 1) / 2 + 1;
    n->pool_w = (S.Wout - 1) / 2 + 1;
    int h = n->pool_h, cin = w0;
    for (int s = 0; s < 4; ++s) {
      const int w = w0 << s;
      for (int j = 0; j < d.blocks[s]; ++j) {
        const int st = (j == 0 && s > 0) ? 2 : 1;
        char p[64];
        snprintf(p, sizeof(p), "enc.s%d.b%d", s, j);
        Block b{};
        // SE-ResNeXt: a bottleneck twice as wide, its 3x3 in `cardinality` groups
        const int m = se ? 2 * w : w, card = se ? d.cardinality : 1;
        if (se && m % card) return fail(PPO_ESHAPE, "bottleneck width %d does not divide into %d groups", m, card);
        b.c1 = add_unit(n, std::string(p) + ".c1", cin, m, 1, 1, 0, h, h);
        b.c2 = add_unit(n, std::string(p) + ".c2", m, m, 3, st, 1, h, h, card);
        if (se && !gconv_supported(geo(n->units[b.c2], 1), card))
          return fail(PPO_ESHAPE, "grouped convolution of %d channels in %d groups not supported", m, card);
        const int ho = n->units[b.c2].Hout;
        b.c3 = add_unit(n, std::string(p) + ".c3", m, 4 * w, 1, 1, 0, ho, ho);
        if (se) {
          const int C = 4 * w;
          if (C % d.se_reduction) return fail(PPO_ESHAPE, "%d channels do not divide by the reduction", C);
          b.R = C / d.se_reduction;
          if ((size_t)(C + b.R + 256) * sizeof(float) > 65536) return fail(PPO_ESHAPE, "squeeze-excite gate too wide");
          b.se1w = add_tensor(n, std::string(p) + ".se1.w", (size_t)b.R * C);
          b.se1b = add_tensor(n, std::string(p) + ".se1.b", b.R);
          b.se2w = add_tensor(n, std::string(p) + ".se2.w", (size_t)C * b.R);
          b.se2b = add_tensor(n, std::string(p) + ".se2.b", C);
          n->se_C = std::max(n->se_C, C);
          n->se_R = std::max(n->se_R, b.R);
        }
        b.ds = (j == 0) ? add_unit(n, std::string(p) + ".ds", cin, 4 * w, 1, st, 0, h, h) : -1;
        if (b.ds >= 0) n->units[b.ds].relu = 0;  // projection shortcut: GroupNorm only
        if (j != 0 && cin != 4 * w) return fail(PPO_ESHAPE, "identity shortcut with a width change");
        n->blocks.push_back(b);
        cin = 4 * w;
        h = ho;
      }
    }
    n->compress = add_unit(n, "enc.compress", cin, d.compress_ch, 3, 1, 1, h, h);
    n->feat_c = d.compress_ch;
    n->feat_hw = h;
  } else {
    return fail(PPO_EINVAL, "unknown trunk");
  }
  n->flat = n->feat_c * n->feat_hw * n->feat_hw;
  n->fc_w = add_tensor(n, "fc.w", (size_t)d.vis_hidden * n->flat);
  n->fc_b = add_tensor(n, "fc.b", d.vis_hidden);
  if (d.goal_mode == PPO_GOAL_POLAR || d.goal_mode == PPO_GOAL_VEC3) {
    n->goal_w = add_tensor(n, "goal.w", (size_t)d.goal_dim * 3);
    n->goal_b = add_tensor(n, "goal.b", d.goal_dim);
  } else if (d.goal_mode == PPO_GOAL_RAW) {
    if (d.goal_dim != 2) return fail(PPO_ESHAPE, "raw goal has goal_dim 2");
  } else if (d.goal_mode == PPO_GOAL_NONE) {
    if (d.goal_dim != 0) return fail(PPO_ESHAPE, "no goal input: goal_dim 0");
  } else {
    return fail(PPO_EINVAL, "unknown goal mode");
  }
  if (d.prev_actions < 0) return fail(PPO_ESHAPE, "negative previous-action count");
  n->emb_rows = (d.prev_actions > 0 ? d.prev_actions : d.num_actions) + 1;
  if (d.prev_act_dim > 0) n->emb = add_tensor(n, "emb", (size_t)n->emb_rows * d.prev_act_dim);
  const int H = d.hidden;
  n->din0 = d.vis_hidden + d.goal_dim + std::max(0, d.prev_act_dim);
  for (int l = 0; l < d.lstm_layers; ++l) {
    const int din = l == 0 ? n->din0 : H;
    char nm[32];
    snprintf(nm, sizeof(nm), "lstm%d.w", l);
    n->lstm_w.push_back(add_tensor(n, nm, (size_t)4 * H * (din + H)));
    snprintf(nm, sizeof(nm), "lstm%d.b", l);
    n->lstm_b.push_back(add_tensor(n, nm, (size_t)4 * H));
  }
  n->head_w = add_tensor(n, "head.w", (size_t)(d.num_actions + 1) * H);
  n->head_b = add_tensor(n, "head.b", d.num_actions + 1);
  return PPO_OK;
}

// ------------------------------------------------------------- workspace
struct Arena {
  size_t off = 0;
  size_t take(size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return o;
  }
};

struct WsLayout {
  // encoder
  size_t x0;                       // [F][h0][w0][in_ch]
  std::vector<size_t> u, a, st;    // per unit
  std::vector<size_t> sey, sez, sea, ses;  // per block with a gate: branch y, pooled z, hidden a1, gate s
  size_t pool, arg;                // resnet max pool out + argmax
  size_t gpart, gbpart, gcoef;     // GroupNorm partials
  size_t ga, gb, gu, gd, gr;       // backward scratch (max unit size)
  size_t dfeat;                    // [F][flat]
  size_t splitk;                   // split-K partial tiles
  // core
  size_t src, wf, mskf, envrow;    // frame map
  size_t z;                        // [F][din0 (+H for act)]
  std::vector<size_t> g, c, cp, hp, hout;  // per layer
  size_t h0g, c0g;                 // gathered start state [L][nb][H]
  size_t zh;                       // act: [B][max(din0, H) + H]
  size_t fstat, dout, dh0, dh1, dG, dG2, dhp, dcp, dvis, whT;
  size_t sync;                     // persistent recurrence barrier words
  size_t wT;                       // one unit's weights reordered for its data gradient
  size_t se_part;                  // squeeze partial sums [kSeMaxSlices][F][widest gate]
  size_t se_da2, se_da1, se_dz;    // gate backward scratch (widest gate)
  size_t total;
};

WsLayout plan(const ppo_net* n, int F, int nb, bool learn) {
  WsLayout w{};
  Arena A;
  const ppo_net_desc& d = n->d;
  const int H = d.hidden, L = d.lstm_layers;
  const size_t f4 = sizeof(float);
  w.x0 = A.take((size_t)F * n->h0 * n->w0 * d.in_ch * f4);
  for (const Unit& u : n->units) {
    const size_t sz = (size_t)F * u.Hout * u.Wout * u.Cout * f4;
    w.u.push_back(A.take(sz));
    w.a.push_back(A.take(sz));
    w.st.push_back(A.take((size_t)F * d.gn_groups * sizeof(float2)));
  }
  w.se_part = A.take((size_t)kSeMaxSlices * F * n->se_C * f4);
  for (const Block& b : n->blocks) {
    const Unit& u3 = n->units[b.c3];
    const bool se = b.R > 0;
    w.sey.push_back(se ? A.take((size_t)F * u3.Hout * u3.Wout * u3.Cout * f4) : 0);
    w.sez.push_back(se ? A.take((size_t)F * u3.Cout * f4) : 0);
    w.sea.push_back(se ? A.take((size_t)F * b.R * f4) : 0);
    w.ses.push_back(se ? A.take((size_t)F * u3.Cout * f4) : 0);
  }
  if (d.trunk == PPO_TRUNK_RESNET || d.trunk == PPO_TRUNK_SERESNEXT) {
    const size_t ps = (size_t)F * n->pool_h * n->pool_w * d.base_width;
    w.pool = A.take(ps * f4);
    w.arg = A.take(ps);
  }
  w.gpart = A.take((size_t)F * n->gn_part * sizeof(float4));
  w.gbpart = A.take((size_t)F * n->gn_part * sizeof(float2));
  w.gcoef = A.take((size_t)F * n->max_G * sizeof(float2));
  w.splitk = A.take(kSplitKBytes);
  w.z = A.take((size_t)F * (n->din0 + H) * f4);
  w.src = A.take((size_t)F * 4);
  w.wf = A.take((size_t)F * 4);
  w.mskf = A.take((size_t)F * 4);
  w.envrow = A.take((size_t)std::max(nb, 1) * 4);
  for (int l = 0; l < L; ++l) {
    w.g.push_back(A.take((size_t)F * 4 * H * f4));
    w.c.push_back(A.take((size_t)F * H * f4));
    w.cp.push_back(A.take((size_t)F * H * f4));
    w.hp.push_back(A.take((size_t)F * H * f4));
    w.hout.push_back(A.take((size_t)F * H * f4));
  }
  w.zh = A.take((size_t)F * (std::max(n->din0, H) + H) * f4);
  if (learn) {
    const size_t mu = (size_t)F * n->max_unit * f4;
    w.ga = A.take(mu);
    w.gb = A.take(mu);
    w.gu = A.take(mu);
    w.gd = A.take(mu);
    w.gr = A.take(mu);
    w.dfeat = A.take((size_t)F * n->flat * f4);
    w.h0g = A.take((size_t)L * std::max(nb, 1) * H * f4);
    w.c0g = A.take((size_t)L * std::max(nb, 1) * H * f4);
    w.fstat = A.take((size_t)F * 8 * f4);
    w.dout = A.take((size_t)F * (d.num_actions + 1) * f4);
    const int wmax = std::max(n->din0, H);
    w.dh0 = A.take((size_t)F * wmax * f4);
    w.dh1 = A.take((size_t)F * wmax * f4);
    w.dG = A.take((size_t)F * 4 * H * f4);
    w.dG2 = A.take(L == 2 ? (size_t)F * 4 * H * f4 : 0);  // layer 0's dG in the two-layer recurrence
    w.dhp = A.take((size_t)std::max(nb, 1) * H * f4);
    w.dcp = A.take((size_t)std::max(nb, 1) * H * f4);
    w.dvis = A.take((size_t)F * d.vis_hidden * f4);
    w.whT = A.take((size_t)4 * H * H * f4);
    w.sync = A.take(kLstmSyncBytes);
    size_t wt_max = 0;
    for (const Unit& u : n->units) wt_max = std::max(wt_max, (size_t)u.Cout * u.K * u.K * u.Cin);
    w.wT = A.take(wt_max * f4);
    w.se_da2 = A.take((size_t)F * n->se_C * f4);
    w.se_da1 = A.take((size_t)F * n->se_R * f4);
    w.se_dz = A.take((size_t)F * n->se_C * f4);
  }
  w.total = A.off;
  return w;
}

// ------------------------------------------------------------ execution
struct Ctx {
  const ppo_net* n;
  const WsLayout* w;
  char* ws;
  const float* params;
  const void* lp;
  float* grad;
  hipStream_t s;
  int F;
  template <typename T = float>
  T* at(size_t off) const {
    return (T*)(ws + off);
  }
  const float* pf(size_t off) const { return params + off; }
  const void* wt(size_t off) const {  // GEMM weight operand
    return n->prec ? (const void*)((const bf16_t*)lp + off) : (const void*)(params + off);
  }
  float* splitk() const { return at(w->splitk); }
  bool keep_u = true;  // store convolution outputs for a backward pass
};

// GroupNorm of a unit in the one-launch form (a workgroup per image and group,
// best when frames are few) or the coalesced partial / finalize / apply form
// (best for large tensors); the element count thresholds (4 M forward, 1 M
// backward, measured) can be tuned with DDPPO_GN_FUSED_MAX / DDPPO_GNB_FUSED_MAX.
bool gn_one_launch(const Ctx& c, const Unit& u, bool bwd = false) {
  const char* e = getenv(bwd ? "DDPPO_GNB_FUSED_MAX" : "DDPPO_GN_FUSED_MAX");
  const long limit = e ? atol(e) : (long)(bwd ? 1 << 20 : 4 << 20);
  const int P = u.Hout * u.Wout, G = c.n->d.gn_groups;
  return gn_fused_npt(P, u.Cout / G) && (long)c.F * P * u.Cout <= limit;
}

// The one-launch GroupNorm reads its convolution's output (in a call that
// keeps outputs for a backward: its split-K partials only) group-major
// (Epi::gm_p), its (image, group) slabs contiguous instead of Cg floats every
// C; in a call that keeps no outputs (act, encode) the stem's GroupNorm also
// writes the max pool of its slab instead of the plain map.  The values are
// the same either way; DDPPO_ACT_FUSED=0 selects the plain forms (tests
// compare the two).
bool act_fused_forms() {
  const char* e = getenv("DDPPO_ACT_FUSED");
  return !(e && e[0] == '0');
}

// Arms the launch timer for the duration of one unit GEMM call when that
// (unit, op) was selected with ppo_gemm_timer_arm.
struct TimerScope {
  TimerScope(const ppo_net* n, int ui, int op) {
    if ((n->timer_unit == ui || n->timer_unit == PPO_TIMER_ALL_UNITS) && n->timer_op == op && n->timer.cap > 0)
      g_gemm_timer = &n->timer;
  }
  ~TimerScope() { g_gemm_timer = nullptr; }
};

ConvGeo geo(const Unit& u, int F) {
  return ConvGeo{F, u.Hin, u.Win, u.Cin, u.Hout, u.Wout, u.Cout, u.K, u.K, u.stride, u.pad};
}

// conv -> GroupNorm (+ residual) (+ ReLU); output NHWC (or channel-major), or
// with pool_out (one-launch form only) its 3x3 / 2 max pool instead.
void unit_fwd(const Ctx& c, int ui, const float* x, const float* res, bool relu, float* out, bool chw,
              float* pool_out = nullptr) {
  const Unit& u = c.n->units[ui];
  const ConvGeo g = geo(u, c.F);
  const int P = u.Hout * u.Wout, G = c.n->d.gn_groups;
  if (gn_one_launch(c, u)) {
    // conv (split-K partials left in place) -> one fused GroupNorm launch
    float* y = c.at(c.w->u[ui]);
    int splits;
    // group-major stores; where a backward reads y in the plain layout, only
    // for split-K partials (the GroupNorm then writes y plainly as it sums them)
    const bool gm = u.groups == 1 && act_fused_forms();
    if (u.groups > 1) {
      launch_gconv_fwd(c.n->prec, g, u.groups, x, c.wt(u.w), y, c.s);
      splits = 1;
    } else {
      TimerScope ts(c.n, ui, 0);
      Epi e = epi(y, u.Cout);
      e.act = c.keep_u ? 0 : 1;
      if (gm) {
        e.gm_p = P;
        e.gm_cg = u.Cout / G;
        e.gm_split_only = c.keep_u ? 1 : 0;
      }
      splits = gemm_conv_fwd(c.n->prec, g, x, c.wt(u.w), e, kSplitKBytes, c.splitk(), c.s, true);
    }
    const float* src = splits > 1 ? c.splitk() : y;
    const bool src_gm = gm && (splits > 1 || !c.keep_u);
    launch_gn_fused(src, splits, (size_t)c.F * P * u.Cout, (splits > 1 && c.keep_u) ? y : nullptr, c.F, P,
                    u.Cout, G, kGnEps, c.pf(u.g), c.pf(u.b), res, relu ? 1 : 0, out, chw ? 1 : 0,
                    c.at<float2>(c.w->st[ui]), c.s, src_gm ? 1 : 0, pool_out, u.Hout, u.Wout);
    return;
  }
  if (u.groups > 1) {
    launch_gconv_fwd(c.n->prec, g, u.groups, x, c.wt(u.w), c.at(c.w->u[ui]), c.s);
  } else {
    TimerScope ts(c.n, ui, 0);
    gemm_conv_fwd(c.n->prec, g, x, c.wt(u.w), epi(c.at(c.w->u[ui]), u.Cout), kSplitKBytes, c.splitk(), c.s);
  }
  launch_gn_forward(c.at(c.w->u[ui]), c.F, u.Hout * u.Wout, u.Cout, c.n->d.gn_groups, kGnEps, c.pf(u.g),
                    c.pf(u.b), res, relu ? 1 : 0, out, chw ? 1 : 0, c.at<float2>(c.w->st[ui]),
                    c.at<float4>(c.w->gpart), u.S, c.s);
}

// A bottleneck's last unit and its projection shortcut in a call that keeps no
// outputs (act, encode): both products deferred (their split-K partials in the
// two halves of the split-K region, group-major), then one GroupNorm launch
// that normalises both and adds the shortcut before the ReLU; the shortcut's
// map is not stored.  Same values as unit_fwd of ds, then of c3 with that residual.
bool pair_fwd_ok(const Ctx& c, int ui, int di) {
  const Unit &u = c.n->units[ui], &d = c.n->units[di];
  return !c.keep_u && act_fused_forms() && u.groups == 1 && d.groups == 1 && u.Cout == d.Cout &&
         u.Hout == d.Hout && u.Wout == d.Wout && gn_one_launch(c, u);
}

void unit_pair_fwd(const Ctx& c, int ui, const float* x, int di, const float* xd, float* out) {
  const Unit &u = c.n->units[ui], &ud = c.n->units[di];
  const int P = u.Hout * u.Wout, G = c.n->d.gn_groups;
  const size_t half = kSplitKBytes / 2;
  float* part_d = (float*)((char*)c.splitk() + half);
  float *y = c.at(c.w->u[ui]), *yd = c.at(c.w->u[di]);
  auto act_epi = [&](float* dst) {
    Epi e = epi(dst, u.Cout);
    e.act = 1;
    e.gm_p = P;
    e.gm_cg = u.Cout / G;
    return e;
  };
  int sd, s3;
  {
    TimerScope ts(c.n, di, 0);
    sd = gemm_conv_fwd(c.n->prec, geo(ud, c.F), xd, c.wt(ud.w), act_epi(yd), half, part_d, c.s, true);
  }
  {
    TimerScope ts(c.n, ui, 0);
    s3 = gemm_conv_fwd(c.n->prec, geo(u, c.F), x, c.wt(u.w), act_epi(y), half, c.splitk(), c.s, true);
  }
  const GnSecond sec{sd > 1 ? part_d : yd, sd, 1, c.pf(ud.g), c.pf(ud.b), c.at<float2>(c.w->st[di])};
  launch_gn_fused(s3 > 1 ? c.splitk() : y, s3, (size_t)c.F * P * u.Cout, nullptr, c.F, P, u.Cout, G, kGnEps,
                  c.pf(u.g), c.pf(u.b), nullptr, 1, out, 0, c.at<float2>(c.w->st[ui]), c.s, 1, nullptr, 0, 0, &sec);
}

// Encoder forward over c.F frames already in x0; returns the flat features
// (channel-major per frame, i.e. [F][flat]).
const float* encoder_fwd(const Ctx& c) {
  const ppo_net* n = c.n;
  const float* x0 = c.at(c.w->x0);
  if (n->d.trunk == PPO_TRUNK_NONE) return x0;  // the input already is [F][flat]
  if (n->d.trunk == PPO_TRUNK_TINY) {
    unit_fwd(c, 0, x0, nullptr, true, c.at(c.w->a[0]), false);
    unit_fwd(c, 1, c.at(c.w->a[0]), nullptr, true, c.at(c.w->a[1]), true);
    return c.at(c.w->a[1]);
  }
  const Unit& S = n->units[n->stem];
  // without a backward the stem's GroupNorm pools its own slab (no plain map,
  // no max-pool launch, no winner indices)
  if (!c.keep_u && act_fused_forms() && gn_one_launch(c, S) && gn_pool_fits(S.Hout * S.Wout, S.Cout / n->d.gn_groups)) {
    unit_fwd(c, n->stem, x0, nullptr, true, c.at(c.w->a[n->stem]), false, c.at(c.w->pool));
  } else {
    unit_fwd(c, n->stem, x0, nullptr, true, c.at(c.w->a[n->stem]), false);
    launch_maxpool_fwd(c.at(c.w->a[n->stem]), c.F, S.Hout, S.Wout, S.Cout, c.at(c.w->pool),
                       c.at<uint8_t>(c.w->arg), c.s);
  }
  const float* x = c.at(c.w->pool);
  for (size_t bi = 0; bi < n->blocks.size(); ++bi) {
    const Block& b = n->blocks[bi];
    unit_fwd(c, b.c1, x, nullptr, true, c.at(c.w->a[b.c1]), false);
    unit_fwd(c, b.c2, c.at(c.w->a[b.c1]), nullptr, true, c.at(c.w->a[b.c2]), false);
    if (b.ds >= 0 && b.R == 0 && pair_fwd_ok(c, b.c3, b.ds)) {
      unit_pair_fwd(c, b.c3, c.at(c.w->a[b.c2]), b.ds, x, c.at(c.w->a[b.c3]));
      x = c.at(c.w->a[b.c3]);
      continue;
    }
    const float* res = x;
    if (b.ds >= 0) {
      unit_fwd(c, b.ds, x, nullptr, false, c.at(c.w->a[b.ds]), false);
      res = c.at(c.w->a[b.ds]);
    }
    if (b.R > 0) {
      // branch y = GN(conv3), gated per channel, then the shortcut and ReLU
      const Unit& u3 = n->units[b.c3];
      unit_fwd(c, b.c3, c.at(c.w->a[b.c2]), nullptr, false, c.at(c.w->sey[bi]), false);
      launch_se_forward(c.at(c.w->sey[bi]), res, c.F, u3.Hout * u3.Wout, u3.Cout, b.R, c.pf(b.se1w), c.pf(b.se1b),
                        c.pf(b.se2w), c.pf(b.se2b), c.at(c.w->se_part), c.at(c.w->sez[bi]), c.at(c.w->sea[bi]),
                        c.at(c.w->ses[bi]), c.at(c.w->a[b.c3]), c.s);
    } else {
      unit_fwd(c, b.c3, c.at(c.w->a[b.c2]), res, true, c.at(c.w->a[b.c3]), false);
    }
    x = c.at(c.w->a[b.c3]);
  }
  unit_fwd(c, n->compress, x, nullptr, true, c.at(c.w->a[n->compress]), true);
  return c.at(c.w->a[n->compress]);
}

// GroupNorm backward + weight gradient + (optional) data gradient of one unit.
//   dout: gradient at the unit's output (layout chw or NHWC); mask_out: the
//   ReLU'd output for the mask (or null); x: the conv input; dx: data gradient
//   out (null = not needed), dx_acc: accumulate into dx; dres: also write the
//   masked output gradient (the residual branch's gradient).
// GroupNorm backward of one unit (fused per image and group when it fits).
void gn_bwd(const Ctx& c, int ui, const float* dout, const float* mask_out, bool chw, float* du, float* dres) {
  const Unit& u = c.n->units[ui];
  const int P = u.Hout * u.Wout, G = c.n->d.gn_groups;
  if (gn_one_launch(c, u, true)) {
    launch_gnb_fused(dout, mask_out, chw ? 1 : 0, c.at(c.w->u[ui]), c.F, P, u.Cout, G, c.at<float2>(c.w->st[ui]),
                     c.pf(u.g), du, dres, c.grad + u.g, c.grad + u.b, c.at<float2>(c.w->gbpart), c.s);
    return;
  }
  launch_gn_backward(dout, mask_out, chw ? 1 : 0, c.at(c.w->u[ui]), c.F, P, u.Cout, G, c.at<float2>(c.w->st[ui]),
                     c.pf(u.g), du, dres, c.grad + u.g, c.grad + u.b, c.at<float2>(c.w->gbpart),
                     c.at<float2>(c.w->gcoef), u.S, c.s);
}

void unit_bwd(const Ctx& c, int ui, const float* dout, const float* mask_out, bool chw, const float* x,
              float* du, float* dx, bool dx_acc, float* dres) {
  const Unit& u = c.n->units[ui];
  const ppo_net* n = c.n;
  const int P = u.Hout * u.Wout;
  gn_bwd(c, ui, dout, mask_out, chw, du, dres);
  const ConvGeo g = geo(u, c.F);
  if (u.groups > 1) {
    launch_gconv_wgrad(n->prec, g, u.groups, x, du, c.grad + u.w, c.splitk(), kSplitKBytes, c.s);
    if (dx) launch_gconv_dgrad(n->prec, g, u.groups, du, c.wt(u.w), dx, dx_acc ? 1 : 0, c.s);
    return;
  }
  const long Kw = (long)u.K * u.K * u.Cin;
  {
    TimerScope ts(n, ui, 2);
    gemm_conv_wgrad(n->prec, g, x, du, epi(c.grad + u.w, (int)Kw), kSplitKBytes, c.splitk(), c.s);
  }
  if (dx) {
    TimerScope ts(n, ui, 1);
    gemm_conv_dgrad(n->prec, g, du, c.wt(u.w), c.at<void>(c.w->wT), epi(dx, u.Cin, nullptr, 0, dx_acc ? 1 : 0),
                    kSplitKBytes, c.splitk(), c.s);
  }
}

void encoder_bwd(const Ctx& c, const float* dfeat) {
  const ppo_net* n = c.n;
  if (n->d.trunk == PPO_TRUNK_NONE) return;
  const WsLayout& w = *c.w;
  const float* x0 = c.at(w.x0);
  float *GA = c.at(w.ga), *GB = c.at(w.gb), *GU = c.at(w.gu), *GD = c.at(w.gd), *GR = c.at(w.gr);
  if (n->d.trunk == PPO_TRUNK_TINY) {
    unit_bwd(c, 1, dfeat, c.at(w.a[1]), true, c.at(w.a[0]), GU, GD, false, nullptr);
    unit_bwd(c, 0, GD, c.at(w.a[0]), false, x0, GU, nullptr, false, nullptr);
    return;
  }
  // compress: input = last block output
  const Block& last = n->blocks.back();
  unit_bwd(c, n->compress, dfeat, c.at(w.a[n->compress]), true, c.at(w.a[last.c3]), GU, GA, false,
           nullptr);
  for (int bi = (int)n->blocks.size() - 1; bi >= 0; --bi) {
    const Block& b = n->blocks[bi];
    const float* xin = bi == 0 ? c.at(w.pool) : c.at(w.a[n->blocks[bi - 1].c3]);
    // GA: gradient at the block output (before its ReLU mask)
    float* dres = b.ds >= 0 ? GR : GB;  // identity: the shortcut gradient seeds dX
    if (b.R > 0) {
      // gate backward: the masked gradient to the shortcut (dres), the branch's into GA
      const Unit& u3 = n->units[b.c3];
      launch_se_backward(GA, c.at(w.a[b.c3]), c.at(w.sey[bi]), c.at(w.sez[bi]), c.at(w.sea[bi]), c.at(w.ses[bi]),
                         c.F, u3.Hout * u3.Wout, u3.Cout, b.R, c.pf(b.se1w), c.pf(b.se2w), dres, c.at(w.se_part),
                         c.at(w.se_da2), c.at(w.se_da1), c.at(w.se_dz), c.grad + b.se1w, c.grad + b.se1b,
                         c.grad + b.se2w, c.grad + b.se2b, GA, c.s);
      unit_bwd(c, b.c3, GA, nullptr, false, c.at(w.a[b.c2]), GU, GD, false, nullptr);
    } else {
      unit_bwd(c, b.c3, GA, c.at(w.a[b.c3]), false, c.at(w.a[b.c2]), GU, GD, false, dres);
    }
    unit_bwd(c, b.c2, GD, c.at(w.a[b.c2]), false, c.at(w.a[b.c1]), GU, GD, false, nullptr);
    if (b.ds >= 0) {
      // c1 first (its du must not be overwritten before its data gradient)
      const Unit& u1 = n->units[b.c1];
      gn_bwd(c, b.c1, GD, c.at(w.a[b.c1]), false, GU, nullptr);
      const ConvGeo g1 = geo(u1, c.F);
      const long K1 = (long)u1.Cin;
      {
        TimerScope ts(n, b.c1, 2);
        gemm_conv_wgrad(n->prec, g1, xin, GU, epi(c.grad + u1.w, (int)K1), kSplitKBytes, c.splitk(), c.s);
      }
      // projection shortcut: writes dX, then c1's data gradient accumulates
      unit_bwd(c, b.ds, GR, nullptr, false, xin, GD, GB, false, nullptr);
      TimerScope ts(n, b.c1, 1);
      gemm_conv_dgrad(n->prec, g1, GU, c.wt(u1.w), c.at<void>(w.wT), epi(GB, u1.Cin, nullptr, 0, 1),
                      kSplitKBytes, c.splitk(), c.s);
    } else {
      unit_bwd(c, b.c1, GD, c.at(w.a[b.c1]), false, xin, GU, GB, true, nullptr);
    }
    std::swap(GA, GB);
  }
  // GA = gradient at the max pool output
  const Unit& S = n->units[n->stem];
  launch_maxpool_bwd(GA, c.at<uint8_t>(w.arg), c.F, S.Hout, S.Wout, S.Cout, GD, c.s);
  unit_bwd(c, n->stem, GD, c.at(w.a[n->stem]), false, x0, GU, nullptr, false, nullptr);
}

hipStream_t strm(void* s) { return (hipStream_t)s; }

// The direct SE-ResNeXt kernels index with 31-bit integers: refuse frame
// counts whose tensors would not fit.
ppo_status check_frames(const ppo_net* n, int F) {
  for (const Unit& u : n->units)
    if (u.groups > 1 && !gconv_fits(geo(u, F))) return fail(PPO_ESHAPE, "%d frames exceed the grouped kernels' indexing", F);
  for (const Block& b : n->blocks)
    if (b.R > 0 && (long)F * n->units[b.c3].Hout * n->units[b.c3].Wout * n->units[b.c3].Cout >= (1L << 31))
      return fail(PPO_ESHAPE, "%d frames exceed the squeeze-excite kernels' indexing", F);
  return PPO_OK;
}

ppo_status check_launch() {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(PPO_EDEVICE, "HIP launch failed: %s", hipGetErrorString(e));
  return PPO_OK;
}

bool al256(const void* p) { return (((uintptr_t)p) & 255) == 0; }

}  // namespace

// ===================================================================== ABI
namespace {

// Static scratch of ppo_loss_head_noalloc: the loss head's workspace for up
// to kNoAllocFrames frames and kMaxMbEnvs envs, resident on every device the
// library runs on until the process ends.  Host code never passes the
// array's name to a kernel: it passes the device address that
// hipGetSymbolAddress returns for the current device (static_scratch).
constexpr int kNoAllocFrames = 32768;
constexpr size_t kNoAllocBytes =
    4 * (((size_t)kNoAllocFrames * 4 + 255) / 256 * 256) + (size_t)kMaxMbEnvs * 4 +
    ((size_t)kNoAllocFrames * 8 * sizeof(float) + 255) / 256 * 256;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch`, looked up once per device.
ppo_status static_scratch(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return fail(PPO_EDEVICE, "no current HIP device");
  }
  if (dev < 0 || dev >= kMaxDevices) return fail(PPO_EUNSUPPORTED, "device index %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(PPO_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return PPO_OK;
}

}  // namespace

extern "C" {

const char* ppo_last_error(void) { return g_err.c_str(); }

// The kernels are built for gfx950 only: a visible current device of another
// architecture is refused.  With no device visible the host-side plan is
// still built (sizes, tensor offsets); compute calls then fail at launch.
ppo_status check_device() {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count == 0) {
    (void)hipGetLastError();
    return PPO_OK;
  }
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return fail(PPO_EDEVICE, "cannot query the current HIP device");
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(PPO_EUNSUPPORTED, "device %d is %s; the library's kernels are built for gfx950", dev,
                prop.gcnArchName);
  return PPO_OK;
}

ppo_status ppo_net_create(const ppo_net_desc* desc, ppo_net** out) {
  if (!desc || !out) return fail(PPO_EINVAL, "null argument");
  *out = nullptr;
  const ppo_status dv = check_device();
  if (dv != PPO_OK) return dv;
  ppo_net* n = new (std::nothrow) ppo_net();
  if (!n) return fail(PPO_EINVAL, "out of host memory");
  n->d = *desc;
  const ppo_status st = build(n);
  if (st != PPO_OK) {
    delete n;
    return st;
  }
  *out = n;
  return PPO_OK;
}

// Waits for the device, then destroys the graphs (none may be in flight).
static int collect_drop(ppo_net* net, size_t keep) {
  if (net->graph_order.size() <= keep) return 0;
  (void)hipDeviceSynchronize();
  int n = 0;
  while (net->graph_order.size() > keep) {
    auto it = net->graphs.find(net->graph_order.front());
    if (it != net->graphs.end()) {
      (void)hipGraphExecDestroy(it->second);
      net->graphs.erase(it);
      ++n;
    }
    net->graph_order.pop_front();
  }
  return n;
}

void ppo_net_destroy(ppo_net* net) {
  if (!net) return;
  collect_drop(net, 0);
  if (net->cap_stream) (void)hipStreamDestroy(net->cap_stream);
  for (hipEvent_t e : net->timer_ev)
    if (e) (void)hipEventDestroy(e);
  delete net;
}

size_t ppo_param_count(const ppo_net* net) { return net ? net->P : 0; }

ppo_status ppo_param_tensor(const ppo_net* net, int i, const char** name, size_t* offset, size_t* count) {
  if (!net || i < 0 || i >= (int)net->tensors.size()) return fail(PPO_EINVAL, "tensor index out of range");
  if (name) *name = net->tensors[i].name.c_str();
  if (offset) *offset = net->tensors[i].off;
  if (count) *count = net->tensors[i].count;
  return PPO_OK;
}

// Workspace of ppo_loss_head: the frame map and the per-frame loss terms.
struct LossWs {
  size_t src, wf, mskf, envrow, fstat, total;
};
LossWs plan_loss(int F, int nb) {
  Arena A;
  LossWs w{};
  w.src = A.take((size_t)F * 4);
  w.wf = A.take((size_t)F * 4);
  w.mskf = A.take((size_t)F * 4);
  w.envrow = A.take((size_t)std::max(nb, 1) * 4);
  w.fstat = A.take((size_t)F * 8 * sizeof(float));
  w.total = A.off;
  return w;
}

ppo_status ppo_workspace_size(const ppo_net* net, int op, int max_frames, int max_envs, size_t* bytes) {
  if (!net || !bytes) return fail(PPO_EINVAL, "null argument");
  if (max_frames <= 0 || (op != PPO_OP_ACT && (max_envs <= 0 || max_envs > kMaxMbEnvs)))
    return fail(PPO_ESHAPE, "bad max_frames / max_envs");
  if (op == PPO_OP_LOSS) {
    *bytes = plan_loss(max_frames, max_envs).total;
    return PPO_OK;
  }
  if (op != PPO_OP_ACT && op != PPO_OP_LEARN) return fail(PPO_EINVAL, "unknown op");
  *bytes = plan(net, max_frames, max_envs, op == PPO_OP_LEARN).total;
  return PPO_OK;
}

// Host-side checks of one ppo_act call, before any launch.
static ppo_status act_check(const ppo_net* net, const ppo_act_io* io, const void* ws, size_t ws_bytes) {
  const ppo_net_desc& d = net->d;
  const int B = io->batch;
  if (B <= 0) return fail(PPO_ESHAPE, "batch must be positive");
  if (!io->obs || (!io->goal && d.goal_mode != PPO_GOAL_NONE) || !io->mask || !io->h_in || !io->c_in || !io->u ||
      !io->params ||
      !io->action || !io->logp || !io->value || !io->h_out || !io->c_out ||
      (d.prev_act_dim > 0 && !io->prev_action) || (net->prec && !io->params_lp))
    return fail(PPO_EINVAL, "null pointer in ppo_act_io");
  if (io->state_rows > 0 && io->state_rows < B) return fail(PPO_ESHAPE, "state_rows < batch");
  if (const ppo_status fs = check_frames(net, B); fs != PPO_OK) return fs;
  const size_t need = plan(net, B, 1, false).total;
  if (!ws || ws_bytes < need) return fail(PPO_EWORKSPACE, "workspace needs %zu bytes", need);
  if (!al256(ws)) return fail(PPO_EWORKSPACE, "workspace must be 256-byte aligned");
  return PPO_OK;
}

ppo_status ppo_act(ppo_net* net, const ppo_act_io* io, void* ws, size_t ws_bytes, void* stream) {
  TuneScope tsc(net);
  if (!net || !io) return fail(PPO_EINVAL, "null argument");
  if (const ppo_status cs = act_check(net, io, ws, ws_bytes); cs != PPO_OK) return cs;
  const ppo_net_desc& d = net->d;
  const int B = io->batch;
  const int SR = io->state_rows > 0 ? io->state_rows : B;
  const WsLayout w = plan(net, B, 1, false);
  const int H = d.hidden, L = d.lstm_layers, A = d.num_actions;
  bool fused = L <= 2;
  for (int l = 0; l < L; ++l) fused = fused && act_layer_supported(l == 0 ? net->din0 : H, H, B);
  hipStream_t s = strm(stream);
  Ctx c{net, &w, (char*)ws, io->params, io->params_lp, nullptr, s, B};
  c.keep_u = false;
  // frames -> encoder -> features
  launch_prep(io->obs, d.trunk == PPO_TRUNK_NONE ? 0 : net->prec, nullptr, B, d.in_ch, d.in_hw, d.in_hw, d.avgpool,
              c.at(w.x0), s);
  const float* feat = encoder_fwd(c);
  // layer-0 input [B][din0 + H] = [relu(FC(feat)) | goal | emb | mask*h0]
  const int ld0 = net->din0 + H;
  float* zh = c.at(w.zh);
  gemm_dense(net->prec, false, false, feat, net->flat, c.wt(net->fc_w), net->prec == 1, net->flat, B,
             d.vis_hidden, net->flat, epi(zh, ld0, c.pf(net->fc_b), 1),
             false, kSplitKBytes, c.splitk(), s);
  const int gmode = d.goal_mode;  // goal kernels: 0 raw, 1 polar, 2 3-vector, 3 none
  const bool polar = gmode == PPO_GOAL_POLAR || gmode == PPO_GOAL_VEC3;  // a goal FC exists
  if (fused) {
    // goal / embedding inputs and every layer's masked state in one launch (all
    // of h_in, c_in read before any output is written), then one launch per
    // layer; the masked copies use the layer-0 gate slab (4 B H floats)
    float* hm = c.at(w.g[0]);
    float* cm = hm + (size_t)L * B * H;
    launch_act_core_prep(io->goal, io->prev_action, io->mask, B, gmode, d.goal_dim,
                         polar ? c.pf(net->goal_w) : nullptr, polar ? c.pf(net->goal_b) : nullptr,
                         std::max(0, d.prev_act_dim), d.prev_act_dim > 0 ? c.pf(net->emb) : nullptr, zh, ld0,
                         d.vis_hidden, io->h_in, io->c_in, L, SR, H, hm, cm, s);
    for (int l = 0; l < L; ++l) {
      const int din = l == 0 ? net->din0 : H;
      const float* X = l == 0 ? zh : io->h_out + (size_t)(l - 1) * SR * H;
      launch_lstm_act_layer(net->prec, X, l == 0 ? ld0 : H, din, hm + (size_t)l * B * H, cm + (size_t)l * B * H,
                            c.wt(net->lstm_w[l]), din + H, c.pf(net->lstm_b[l]), B, H,
                            io->h_out + (size_t)l * SR * H, io->c_out + (size_t)l * SR * H, io->active, s);
    }
    launch_act_head(io->h_out + (size_t)(L - 1) * SR * H, B, H, A, c.pf(net->head_w), c.pf(net->head_b),
                    io->u, io->action, io->logp, io->value, io->logits, io->active, s);
    return check_launch();
  }
  launch_embed_fwd(io->goal, io->prev_action, io->mask, nullptr, B, gmode,
                   d.goal_dim, polar ? c.pf(net->goal_w) : nullptr,
                   polar ? c.pf(net->goal_b) : nullptr, std::max(0, d.prev_act_dim),
                   d.prev_act_dim > 0 ? c.pf(net->emb) : nullptr, zh, ld0, d.vis_hidden, s);
  // masked recurrent state of every layer, read before any output is written
  std::vector<float*> zl(L), cpl(L);
  for (int l = 0; l < L; ++l) {
    const int din = l == 0 ? net->din0 : H;
    zl[l] = l == 0 ? zh : c.at(w.g[l]);  // layer l>0 input buffer [B][2H] (reuses its gate slab)
    cpl[l] = c.at(w.cp[l]);
    launch_mask_state(io->h_in + (size_t)l * SR * H, io->c_in + (size_t)l * SR * H, io->mask, B, H,
                      zl[l] + din, din + H, cpl[l], s);
  }
  // with a device row count, every layer's h and c go to workspace rows first
  // and only the active rows are copied out
  const bool masked = io->active != nullptr;
  for (int l = 0; l < L; ++l) {
    const int din = l == 0 ? net->din0 : H;
    const bool top = l == L - 1;
    float* hdst = top ? (masked ? c.at(w.hout[l]) : io->h_out + (size_t)l * SR * H) : zl[l + 1];
    float* cdst = masked ? c.at(w.c[l]) : io->c_out + (size_t)l * SR * H;
    const int ldh = top ? H : 2 * H;
    // gates = [x | m h] [W_ih | W_hh]^T + b and the cell, in one launch
    launch_lstm_step_fwd(net->prec, zl[l], din + H, din + H, c.wt(net->lstm_w[l]), din + H, nullptr,
                         c.pf(net->lstm_b[l]), cpl[l], B, H, nullptr, hdst, ldh, cdst, nullptr, 0, nullptr, 0,
                         nullptr, s);
    if (!top || masked) launch_copy2d(hdst, ldh, B, H, io->h_out + (size_t)l * SR * H, H, s, io->active);
    if (masked) launch_copy2d(cdst, H, B, H, io->c_out + (size_t)l * SR * H, H, s, io->active);
  }
  launch_act_head(io->h_out + (size_t)(L - 1) * SR * H, B, H, A, c.pf(net->head_w), c.pf(net->head_b),
                  io->u, io->action, io->logp, io->value, io->logits, io->active, s);
  return check_launch();
}

// Step t's ppo_act arguments inside a rollout's buffers (rows: its batch).
static ppo_act_io collect_step(const ppo_net* net, const ppo_collect_io* io, int t, int rows, bool trim) {
  const ppo_net_desc& d = net->d;
  const size_t N = (size_t)io->N;
  const size_t esz = net->prec && d.trunk != PPO_TRUNK_NONE ? 2 : 4;
  const size_t frame = (size_t)d.in_ch * d.in_hw * d.in_hw;
  const size_t gw = d.goal_mode == PPO_GOAL_NONE ? 0 : d.goal_mode == PPO_GOAL_VEC3 ? 3 : 2;
  const size_t state = (size_t)d.lstm_layers * N * d.hidden;
  ppo_act_io a{};
  a.batch = rows;
  a.state_rows = io->N;
  a.obs = (const char*)io->obs + (size_t)t * N * frame * esz;
  a.goal = io->goal ? io->goal + (size_t)t * N * gw : nullptr;
  a.prev_action = io->actions + (size_t)t * N;
  a.mask = io->mask + (size_t)t * N;
  a.h_in = io->h_hist + (size_t)t * state;
  a.c_in = io->c_hist + (size_t)t * state;
  a.u = io->u + (size_t)t * N;
  a.params = io->params;
  a.params_lp = io->params_lp;
  a.action = io->actions + (size_t)(t + 1) * N;
  a.logp = io->logp + (size_t)t * N;
  a.value = io->value + (size_t)t * N;
  a.h_out = t < io->T ? io->h_hist + (size_t)(t + 1) * state : io->h_last;
  a.c_out = t < io->T ? io->c_hist + (size_t)(t + 1) * state : io->c_last;
  a.logits = nullptr;
  a.active = trim || !io->active ? nullptr : io->active + t;
  return a;
}

// The steps of one ppo_collect call, launched on s (rows[t]: step t's batch;
// the steps stop at the first with none).
static ppo_status collect_run(ppo_net* net, const ppo_collect_io* io, const std::vector<int>& rows, bool trim,
                              void* ws, size_t ws_bytes, hipStream_t s) {
  for (int t = io->t_begin; t < io->t_end && rows[t] > 0; ++t) {
    const ppo_act_io a = collect_step(net, io, t, rows[t], trim);
    if (const ppo_status st = ppo_act(net, &a, ws, ws_bytes, s); st != PPO_OK) return st;
  }
  return PPO_OK;
}

constexpr size_t kMaxCollectGraphs = 1024;

ppo_status ppo_collect(ppo_net* net, const ppo_collect_io* io, int flags, void* ws, size_t ws_bytes,
                       void* stream) {
  if (!net || !io) return fail(PPO_EINVAL, "null argument");
  const ppo_net_desc& d = net->d;
  const int T = io->T, N = io->N;
  if (T < 0 || N <= 0) return fail(PPO_ESHAPE, "need T >= 0 and N > 0");
  if (io->t_begin < 0 || io->t_begin > io->t_end || io->t_end > T + 1)
    return fail(PPO_ESHAPE, "step range [%d, %d) outside [0, %d]", io->t_begin, io->t_end, T + 1);
  if (!io->actions || !io->h_hist || !io->c_hist || !io->h_last || !io->c_last)
    return fail(PPO_EINVAL, "null pointer in ppo_collect_io");
  if (flags & ~(PPO_COLLECT_GRAPH | PPO_COLLECT_TRIM)) return fail(PPO_EINVAL, "unknown flags %d", flags);
  const bool trim = flags & PPO_COLLECT_TRIM;
  // every step's batch (host), and the checks of the largest step's call
  std::vector<int> rows(T + 1, N);
  if (trim && io->lengths) {
    for (int n = 0; n < N; ++n) {
      if (io->lengths[n] < 0 || io->lengths[n] > T) return fail(PPO_ESHAPE, "length %d outside [0, %d]", io->lengths[n], T);
      if (n > 0 && io->lengths[n] > io->lengths[n - 1])
        return fail(PPO_ESHAPE, "lengths must be non-increasing (envs ordered longest first)");
    }
    for (int t = 0; t <= T; ++t) {
      int b = 0;
      while (b < N && io->lengths[b] >= t) ++b;
      rows[t] = b;
    }
  }
  if (io->t_begin == io->t_end) return PPO_OK;
  {
    const ppo_act_io a = collect_step(net, io, io->t_begin, N, trim);
    if (const ppo_status cs = act_check(net, &a, ws, ws_bytes); cs != PPO_OK) return cs;
  }
  hipStream_t s = strm(stream);
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess) return check_launch();
  if (!(flags & PPO_COLLECT_GRAPH) || cs != hipStreamCaptureStatusNone)
    return collect_run(net, io, rows, trim, ws, ws_bytes, s);
  // the graph of this argument set: every field, the workspace, the flags, the lengths
  std::string key;
  auto put = [&key](const void* p, size_t n) { key.append((const char*)p, n); };
  const void* ptrs[] = {io->obs, io->goal, io->mask, io->u, io->active, io->params, io->params_lp, io->actions,
                        io->logp, io->value, io->h_hist, io->c_hist, io->h_last, io->c_last, ws};
  const int ints[] = {T, N, io->t_begin, io->t_end, flags};
  put(ptrs, sizeof(ptrs));
  put(ints, sizeof(ints));
  put(&ws_bytes, sizeof(ws_bytes));
  if (trim) put(rows.data(), rows.size() * sizeof(int));
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return check_launch();
  if (net->cap_stream && net->cap_device != dev)
    return fail(PPO_EINVAL, "the net's act graphs live on device %d, not %d", net->cap_device, dev);
  auto hit = net->graphs.find(key);
  if (hit != net->graphs.end()) {
    if (hipGraphLaunch(hit->second, s) != hipSuccess) return check_launch();
    return PPO_OK;
  }
  // first call: eager steps (their results stand), then capture on the private stream
  if (const ppo_status st = collect_run(net, io, rows, trim, ws, ws_bytes, s); st != PPO_OK) return st;
  if (!net->cap_stream) {
    if (hipStreamCreateWithFlags(&net->cap_stream, hipStreamNonBlocking) != hipSuccess) return check_launch();
    net->cap_device = dev;
  }
  collect_drop(net, kMaxCollectGraphs - 1);
  // the launch timer stays out of captured graphs (its events are re-armed and destroyed by the host)
  const int tu = net->timer_unit;
  net->timer_unit = -1;
  hipGraph_t g = nullptr;
  ppo_status st = PPO_OK;
  if (hipStreamBeginCapture(net->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    st = check_launch();
  } else {
    st = collect_run(net, io, rows, trim, ws, ws_bytes, net->cap_stream);
    const hipError_t e = hipStreamEndCapture(net->cap_stream, &g);
    if (st == PPO_OK && (e != hipSuccess || !g)) st = fail(PPO_EDEVICE, "act graph capture failed: %s", hipGetErrorString(e));
  }
  net->timer_unit = tu;
  hipGraphExec_t exec = nullptr;
  if (st == PPO_OK && hipGraphInstantiate(&exec, g, nullptr, nullptr, 0) != hipSuccess)
    st = fail(PPO_EDEVICE, "act graph instantiation failed: %s", hipGetErrorString(hipGetLastError()));
  if (g) (void)hipGraphDestroy(g);
  (void)hipGetLastError();
  if (st != PPO_OK) return st;
  net->graphs.emplace(key, exec);
  net->graph_order.push_back(key);
  return PPO_OK;
}

int ppo_collect_clear(ppo_net* net) { return net ? collect_drop(net, 0) : 0; }

int ppo_collect_graph_count(const ppo_net* net) { return net ? (int)net->graphs.size() : 0; }

ppo_status ppo_gae(const float* rew, const float* val, const uint8_t* done, const int32_t* len, int T,
                   int N, float gamma, float lambda, float* adv, float* ret, double* adv_stats,
                   void* stream) {
  if (!rew || !val || !done || !adv || !ret) return fail(PPO_EINVAL, "null argument");
  if (T <= 0 || N <= 0) return fail(PPO_ESHAPE, "T and N must be positive");
  if (!(gamma >= 0.f && gamma <= 1.f) || !(lambda >= 0.f && lambda <= 1.f))
    return fail(PPO_EINVAL, "gamma and lambda must lie in [0, 1]");
  launch_gae(rew, val, done, len, T, N, gamma, lambda, adv, ret, adv_stats, strm(stream));
  return check_launch();
}

}  // extern "C"

namespace {

// Minibatch schedule: envs sorted by length (longest first, stable), frames
// packed time-major; step t holds the first act[t] envs at frames off[t]...
struct Sched {
  MapArgs m;
  int F = 0, TB = 0;
  std::vector<int> act, off;
};

// Packing of a minibatch (envs longest first, frames time-major).  inputs:
// also require the policy inputs (frames, goal, state, parameters).
ppo_status schedule(const ppo_net* net, const ppo_batch* b, Sched& S, bool inputs = true, bool per_step = true) {
  const ppo_net_desc& d = net->d;
  if (!b->env_ids || !b->mask ||
      (inputs && (!b->obs || (!b->goal && d.goal_mode != PPO_GOAL_NONE) || !b->h0 || !b->c0 || !b->params ||
                  (net->prec && !b->params_lp) ||
                  (d.prev_act_dim > 0 && !b->prev_action))))
    return fail(PPO_EINVAL, "null pointer in ppo_batch");
  if (b->T <= 0 || b->N <= 0 || b->nb <= 0 || b->nb > b->N || b->nb > kMaxMbEnvs)
    return fail(PPO_ESHAPE, "bad T / N / nb");
  S.m = MapArgs{};
  S.m.nb = b->nb;
  S.m.N = b->N;
  S.m.T = b->T;
  std::vector<std::pair<int, int>> order;
  for (int j = 0; j < b->nb; ++j) {
    const int e = b->env_ids[j];
    if (e < 0 || e >= b->N) return fail(PPO_ESHAPE, "env id %d out of range", e);
    const int len = b->lengths ? b->lengths[e] : b->T;
    if (len < 1 || len > b->T) return fail(PPO_ESHAPE, "length %d of env %d outside 1..T", len, e);
    order.push_back({len, e});
  }
  std::stable_sort(order.begin(), order.end(),
                   [](const std::pair<int, int>& x, const std::pair<int, int>& y) { return x.first > y.first; });
  S.F = 0;
  for (int j = 0; j < b->nb; ++j) {
    S.m.env[j] = order[j].second;
    S.m.len[j] = order[j].first;
    S.F += order[j].first;
  }
  S.m.F = S.F;
  S.TB = S.m.len[0];
  if (!per_step) return PPO_OK;  // frame map only (no host allocation)
  S.act.assign(S.TB + 1, 0);
  S.off.assign(S.TB + 1, 0);
  for (int t = 0; t < S.TB; ++t) {
    for (int j = 0; j < b->nb; ++j) S.act[t] += (S.m.len[j] > t);
    S.off[t + 1] = S.off[t] + S.act[t];
  }
  return PPO_OK;
}

// Forward over every frame of the minibatch: encoder, visual FC, goal and
// previous-action inputs, the LSTM over time.  Returns the flat features;
// the top LSTM output is left in the layer's hout buffer.
const float* learner_fwd(const Ctx& c, const ppo_batch* b, const Sched& S) {
  const ppo_net* net = c.n;
  const ppo_net_desc& d = net->d;
  const WsLayout& w = *c.w;
  hipStream_t s = c.s;
  const int F = S.F, TB = S.TB;
  const std::vector<int>& act = S.act;
  const std::vector<int>& off = S.off;
  const int H = d.hidden, L = d.lstm_layers, nb = b->nb;
  const int32_t* src = c.at<int32_t>(w.src);
  const float* mskf = c.at(w.mskf);
  const int32_t* envrow = c.at<int32_t>(w.envrow);
  launch_frame_map(S.m, b->mask, c.at<int32_t>(w.src), c.at(w.wf), c.at(w.mskf), c.at<int32_t>(w.envrow), s);
  launch_lstm_clear_error(c.at<unsigned>(w.sync), s);
  launch_gather_state(b->h0, L, b->N, nb, H, envrow, c.at(w.h0g), s);
  launch_gather_state(b->c0, L, b->N, nb, H, envrow, c.at(w.c0g), s);

  launch_prep(b->obs, d.trunk == PPO_TRUNK_NONE ? 0 : net->prec, src, F, d.in_ch, d.in_hw, d.in_hw, d.avgpool,
              c.at(w.x0), s);
  const float* feat = encoder_fwd(c);
  const int D0 = net->din0;
  float* Z = c.at(w.z);
  gemm_dense(net->prec, false, false, feat, net->flat, c.wt(net->fc_w), net->prec == 1, net->flat, F,
             d.vis_hidden, net->flat, epi(Z, D0, c.pf(net->fc_b), 1), false, kSplitKBytes, c.splitk(), s);
  const int gmode = d.goal_mode;  // goal kernels: 0 raw, 1 polar, 2 3-vector, 3 none
  const bool polar = gmode == PPO_GOAL_POLAR || gmode == PPO_GOAL_VEC3;  // a goal FC exists
  const int E = std::max(0, d.prev_act_dim);
  launch_embed_fwd(b->goal, b->prev_action, b->mask, src, F, gmode, d.goal_dim,
                   polar ? c.pf(net->goal_w) : nullptr, polar ? c.pf(net->goal_b) : nullptr, E,
                   E ? c.pf(net->emb) : nullptr, Z, D0, d.vis_hidden, s);
  if (L == 2) {
    // both layers in one pipelined launch: only layer 0's input projection runs as a product
    const size_t w0 = net->lstm_w[0], w1 = net->lstm_w[1];
    gemm_dense(net->prec, false, false, Z, D0, c.wt(w0), net->prec == 1, D0 + H, F, 4 * H, D0,
               epi(c.at(w.g[0]), 4 * H, c.pf(net->lstm_b[0])), false, kSplitKBytes, c.splitk(), s);
    for (int l = 0; l < 2; ++l)
      launch_mask_state(c.at(w.h0g) + (size_t)l * nb * H, c.at(w.c0g) + (size_t)l * nb * H, mskf, act[0], H,
                        c.at(w.hp[l]), H, c.at(w.cp[l]), s);
    if (launch_lstm_seq2_fwd(net->prec, S.m, TB, H, c.wt(w0 + D0), D0 + H,
                             c.wt(w1), c.pf(net->lstm_b[1]), c.at(w.g[0]), c.at(w.hp[0]), c.at(w.cp[0]),
                             c.at(w.c[0]), c.at(w.hout[0]), c.at(w.g[1]), c.at(w.hp[1]), c.at(w.cp[1]),
                             c.at(w.c[1]), c.at(w.hout[1]), mskf, c.at<unsigned>(w.sync), s) == 0)
      return feat;
  }
  for (int l = 0; l < L; ++l) {
    const int din = l == 0 ? D0 : H;
    const float* X = l == 0 ? Z : c.at(w.hout[l - 1]);
    const size_t wl = net->lstm_w[l];
    float *G = c.at(w.g[l]), *HP = c.at(w.hp[l]), *CP = c.at(w.cp[l]), *Cs = c.at(w.c[l]),
          *Ho = c.at(w.hout[l]);
    // input projection of every frame at once
    gemm_dense(net->prec, false, false, X, din, c.wt(wl), net->prec == 1, din + H, F, 4 * H, din,
               epi(G, 4 * H, c.pf(net->lstm_b[l])), false, kSplitKBytes, c.splitk(), s);
    launch_mask_state(c.at(w.h0g) + (size_t)l * nb * H, c.at(w.c0g) + (size_t)l * nb * H, mskf, act[0], H,
                      HP, H, CP, s);
    const void* whh = net->prec ? (const void*)((const bf16_t*)b->params_lp + wl + din)
                                : (const void*)(b->params + wl + din);
    if (launch_lstm_seq_fwd(net->prec, S.m, TB, H, whh, din + H, G, HP, CP, Cs, Ho, H, mskf,
                            c.at<unsigned>(w.sync), s) == 0)
      continue;
    for (int t = 0; t < TB; ++t) {
      // gates_t = (x_t W_ih^T + b) + (m_t h_{t-1}) W_hh^T, then the cell (activations overwrite G)
      const size_t r0 = off[t];
      const bool more = t + 1 < TB;
      launch_lstm_step_fwd(net->prec, HP + r0 * H, H, H, whh, din + H, G + r0 * 4 * H, nullptr, CP + r0 * H,
                           act[t], H, G + r0 * 4 * H, Ho + r0 * H, H, Cs + r0 * H,
                           more ? mskf + off[t + 1] : nullptr, more ? act[t + 1] : 0,
                           more ? HP + (size_t)off[t + 1] * H : nullptr, H,
                           more ? CP + (size_t)off[t + 1] * H : nullptr, s);
    }
  }
  return feat;
}

// Backward from dout [F][A+1] (w.dout) and the gradient at the top LSTM
// output (w.dh0), through the LSTM, the FC and input parts and the encoder.
// c.grad null: data gradients only (a frozen net: no parameter gradient, no
// encoder backward); dgoal (3-vector goal mode, or null): the gradient at the
// goal input [F][3] in packed frame order.
void learner_bwd(const Ctx& c, const ppo_batch* b, const Sched& S, const float* feat, float* dgoal = nullptr) {
  const ppo_net* net = c.n;
  const ppo_net_desc& d = net->d;
  const WsLayout& w = *c.w;
  hipStream_t s = c.s;
  float* grad = c.grad;
  const int F = S.F, TB = S.TB;
  const std::vector<int>& act = S.act;
  const std::vector<int>& off = S.off;
  const int H = d.hidden, L = d.lstm_layers, A = d.num_actions;
  const int32_t* src = c.at<int32_t>(w.src);
  const float* mskf = c.at(w.mskf);
  const int D0 = net->din0;
  float* Z = c.at(w.z);
  const int gmode = d.goal_mode;  // goal kernels: 0 raw, 1 polar, 2 3-vector, 3 none
  const bool polar = gmode == PPO_GOAL_POLAR || gmode == PPO_GOAL_VEC3;  // a goal FC exists
  const int E = std::max(0, d.prev_act_dim);
  const float* Htop = c.at(w.hout[L - 1]);
  float* dout = c.at(w.dout);
  float* dH = c.at(w.dh0);
  // the head is float32 in both precisions (forward and its weight gradient)
  if (grad)
    gemm_dense(0, true, true, dout, A + 1, Htop, false, H, A + 1, H, F,
               epi(grad + net->head_w, H), false, kSplitKBytes, c.splitk(), s);
  if (grad)
    launch_colsum(dout, F, A + 1, A + 1, grad + net->head_b, s);
  float* dHn = c.at(w.dh1);
  int l_top = L - 1;
  if (L == 2) {
    // both layers in one pipelined launch; layer 0's input gradient is formed in-kernel
    const size_t w0 = net->lstm_w[0], w1 = net->lstm_w[1];
    float *dG0 = c.at(w.dG2), *dG1 = c.at(w.dG);
    if (launch_lstm_seq2_bwd(net->prec, S.m, TB, H, c.wt(w0 + D0), D0 + H, c.wt(w1), c.at(w.g[0]), c.at(w.cp[0]),
                             c.at(w.c[0]), c.at(w.g[1]), c.at(w.cp[1]), c.at(w.c[1]), dH, dG0, dG1, mskf,
                             c.at<unsigned>(w.sync), s) == 0) {
      const float* H0 = c.at(w.hout[0]);
      if (grad)
        gemm_dense(net->prec, true, true, dG1, 4 * H, H0, false, H, 4 * H, H, F, epi(grad + w1, 2 * H), true,
                   kSplitKBytes, c.splitk(), s);
      if (grad)
        gemm_dense(net->prec, true, true, dG1, 4 * H, c.at(w.hp[1]), false, H, 4 * H, H, F,
                   epi(grad + w1 + H, 2 * H), true, kSplitKBytes, c.splitk(), s);
      if (grad)
        launch_colsum(dG1, F, 4 * H, 4 * H, grad + net->lstm_b[1], s);
      if (grad)
        gemm_dense(net->prec, true, true, dG0, 4 * H, Z, false, D0, 4 * H, D0, F, epi(grad + w0, D0 + H), true,
                   kSplitKBytes, c.splitk(), s);
      if (grad)
        gemm_dense(net->prec, true, true, dG0, 4 * H, c.at(w.hp[0]), false, H, 4 * H, H, F,
                   epi(grad + w0 + D0, D0 + H), true, kSplitKBytes, c.splitk(), s);
      if (grad)
        launch_colsum(dG0, F, 4 * H, 4 * H, grad + net->lstm_b[0], s);
      gemm_dense(net->prec, false, true, dG0, 4 * H, c.wt(w0), net->prec == 1, D0 + H, F, D0, 4 * H,
                 epi(dHn, D0), true, kSplitKBytes, c.splitk(), s);
      std::swap(dH, dHn);
      l_top = -1;
    }
  }
  for (int l = l_top; l >= 0; --l) {
    const int din = l == 0 ? D0 : H;
    const float* X = l == 0 ? Z : c.at(w.hout[l - 1]);
    const size_t wl = net->lstm_w[l];
    float *G = c.at(w.g[l]), *HP = c.at(w.hp[l]), *CP = c.at(w.cp[l]), *Cs = c.at(w.c[l]);
    float *dG = c.at(w.dG), *dcp = c.at(w.dcp);
    const void* whh = net->prec ? (const void*)((const bf16_t*)b->params_lp + wl + din)
                                : (const void*)(b->params + wl + din);
    void* whT = c.at<void>(w.whT);
    const bool seq = launch_lstm_seq_bwd(net->prec, S.m, TB, H, whh, din + H, G, CP, Cs, dH, H, dG, mskf,
                                         c.at<unsigned>(w.sync), s) == 0;
    if (!seq) launch_transpose_whh(net->prec, whh, din + H, H, whT, s);
    for (int t = seq ? -1 : TB - 1; t >= 0; --t) {
      // dh_t = dH_t + m_{t+1} dG_{t+1} W_hh, dc_t = m_{t+1} dc_{t+1} f_{t+1}; cell backward -> dG_t
      const size_t r0 = off[t];
      const bool more = t + 1 < TB;
      launch_lstm_step_bwd(net->prec, more ? dG + (size_t)off[t + 1] * 4 * H : nullptr, whT,
                           more ? mskf + off[t + 1] : nullptr, more ? act[t + 1] : 0, G + r0 * 4 * H,
                           Cs + r0 * H, CP + r0 * H, dH + r0 * H, H, act[t], H, dG + r0 * 4 * H, dcp, s);
    }
    // weight gradients over all frames
    if (grad)
      gemm_dense(net->prec, true, true, dG, 4 * H, X, false, din, 4 * H, din, F, epi(grad + wl, din + H),
                 true, kSplitKBytes, c.splitk(), s);
    if (grad)
      gemm_dense(net->prec, true, true, dG, 4 * H, HP, false, H, 4 * H, H, F, epi(grad + wl + din, din + H),
                 true, kSplitKBytes, c.splitk(), s);
    if (grad)
      launch_colsum(dG, F, 4 * H, 4 * H, grad + net->lstm_b[l], s);
    // gradient into the layer input
    gemm_dense(net->prec, false, true, dG, 4 * H, c.wt(wl), net->prec == 1, din + H, F, din, 4 * H,
               epi(dHn, din), true, kSplitKBytes, c.splitk(), s);
    std::swap(dH, dHn);
  }
  // dH = gradient at Z [F][D0]
  float* dvis = c.at(w.dvis);
  launch_relu_grad2d(dH, D0, Z, D0, F, d.vis_hidden, dvis, d.vis_hidden, s);
  if (grad)
    launch_embed_bwd(b->goal, b->prev_action, b->mask, src, F, gmode, d.goal_dim, E, net->emb_rows, dH, D0,
                     d.vis_hidden, polar ? grad + net->goal_w : nullptr, polar ? grad + net->goal_b : nullptr,
                     E ? grad + net->emb : nullptr, s);
  if (grad)
    gemm_dense(net->prec, true, true, dvis, d.vis_hidden, feat, false, net->flat, d.vis_hidden, net->flat, F,
               epi(grad + net->fc_w, net->flat), true, kSplitKBytes, c.splitk(), s);
  if (grad)
    launch_colsum(dvis, F, d.vis_hidden, d.vis_hidden, grad + net->fc_b, s);
  if (dgoal) launch_goal_dgrad(dH, D0, d.vis_hidden, F, d.goal_dim, c.pf(net->goal_w), dgoal, s);
  if (!grad || d.trunk == PPO_TRUNK_NONE) return;  // nothing upstream to train
  float* dfeat = c.at(w.dfeat);
  gemm_dense(net->prec, false, true, dvis, d.vis_hidden, c.wt(net->fc_w), net->prec == 1, net->flat, F,
             net->flat, d.vis_hidden, epi(dfeat, net->flat), true, kSplitKBytes, c.splitk(),
             s);
  encoder_bwd(c, dfeat);
}

// The PPO objective on given policy outputs (ppo_loss_head and its variant
// without allocation).  noalloc: the workspace is the static scratch array;
// no host or device allocation on this path.
ppo_status loss_head(ppo_net* net, const ppo_batch* b, const ppo_loss_cfg* cfg, const float* d_loss_scale,
                     const float* logits, const float* values, float* dlogits, float* dvalues, float* stats,
                     float* loss_out, void* ws, size_t ws_bytes, void* stream, bool noalloc) {
  if (!net || !b || !cfg || !logits || !values || !dlogits || !dvalues || !stats)
    return fail(PPO_EINVAL, "null argument");
  if (!b->action || !b->logp_old || !b->adv || !b->ret || (cfg->norm_adv && !cfg->adv_stats))
    return fail(PPO_EINVAL, "null pointer in ppo_batch");
  Sched S;
  const ppo_status st = schedule(net, b, S, false, false);
  if (st != PPO_OK) return st;
  if (noalloc && S.F > kNoAllocFrames)
    return fail(PPO_ESHAPE, "%d frames exceed the %d of the static scratch of ppo_loss_head_noalloc", S.F,
                kNoAllocFrames);
  const LossWs w = plan_loss(S.F, b->nb);
  if (!ws || ws_bytes < w.total) return fail(PPO_EWORKSPACE, "workspace needs %zu bytes", w.total);
  if (!al256(ws)) return fail(PPO_EWORKSPACE, "workspace must be 256-byte aligned");
  hipStream_t s = strm(stream);
  char* base = (char*)ws;
  launch_frame_map(S.m, b->mask, (int32_t*)(base + w.src), (float*)(base + w.wf), (float*)(base + w.mskf),
                   (int32_t*)(base + w.envrow), s);
  launch_loss_terms(logits, values, S.F, net->d.num_actions, (const int32_t*)(base + w.src), b->action,
                    b->logp_old, b->adv, b->ret, (const float*)(base + w.wf), cfg->clip, cfg->value_coef,
                    cfg->entropy_coef, cfg->norm_adv, cfg->adv_stats, net->prec ? d_loss_scale : nullptr,
                    (float*)(base + w.fstat), dlogits, dvalues, stats, loss_out, s);
  return check_launch();
}


}  // namespace

extern "C" {

ppo_status ppo_loss_backward(ppo_net* net, const ppo_batch* b, const ppo_loss_cfg* cfg,
                             const float* d_loss_scale, float* grad, float* stats, void* ws,
                             size_t ws_bytes, void* stream) {
  TuneScope tsc(net);
  if (!net || !b || !cfg || !grad || !stats) return fail(PPO_EINVAL, "null argument");
  if (!b->action || !b->logp_old || !b->adv || !b->ret || (cfg->norm_adv && !cfg->adv_stats))
    return fail(PPO_EINVAL, "null pointer in ppo_batch");
  Sched S;
  const ppo_status st = schedule(net, b, S);
  if (st != PPO_OK) return st;
  const WsLayout w = plan(net, S.F, b->nb, true);
  if (const ppo_status fs = check_frames(net, S.F); fs != PPO_OK) return fs;
  if (!ws || ws_bytes < w.total) return fail(PPO_EWORKSPACE, "workspace needs %zu bytes", w.total);
  if (!al256(ws)) return fail(PPO_EWORKSPACE, "workspace must be 256-byte aligned");
  hipStream_t s = strm(stream);
  Ctx c{net, &w, (char*)ws, b->params, b->params_lp, grad, s, S.F};
  const ppo_net_desc& d = net->d;
  const int H = d.hidden, A = d.num_actions;
  const float* feat = learner_fwd(c, b, S);
  launch_loss_head(c.at(w.hout[d.lstm_layers - 1]), S.F, H, A, c.pf(net->head_w), c.pf(net->head_b),
                   c.at<int32_t>(w.src), b->action, b->logp_old, b->adv, b->ret, c.at(w.wf), cfg->clip,
                   cfg->value_coef, cfg->entropy_coef, cfg->norm_adv, cfg->adv_stats,
                   net->prec ? d_loss_scale : nullptr, c.at(w.fstat), c.at(w.dout), c.at(w.dh0), stats, s);
  learner_bwd(c, b, S, feat);
  return check_launch();
}

ppo_status ppo_policy_forward(ppo_net* net, const ppo_batch* b, float* logits, float* values, int32_t* frame_src,
                              void* ws, size_t ws_bytes, void* stream) {
  TuneScope tsc(net);
  if (!net || !b || !logits || !values) return fail(PPO_EINVAL, "null argument");
  Sched S;
  const ppo_status st = schedule(net, b, S);
  if (st != PPO_OK) return st;
  const WsLayout w = plan(net, S.F, b->nb, true);
  if (const ppo_status fs = check_frames(net, S.F); fs != PPO_OK) return fs;
  if (!ws || ws_bytes < w.total) return fail(PPO_EWORKSPACE, "workspace needs %zu bytes", w.total);
  if (!al256(ws)) return fail(PPO_EWORKSPACE, "workspace must be 256-byte aligned");
  hipStream_t s = strm(stream);
  Ctx c{net, &w, (char*)ws, b->params, b->params_lp, nullptr, s, S.F};
  const ppo_net_desc& d = net->d;
  learner_fwd(c, b, S);
  launch_head_fwd(c.at(w.hout[d.lstm_layers - 1]), S.F, d.hidden, d.num_actions, c.pf(net->head_w),
                  c.pf(net->head_b), logits, values, s);
  if (frame_src) launch_copy_i32(c.at<int32_t>(w.src), S.F, frame_src, s);
  return check_launch();
}

ppo_status ppo_policy_backward(ppo_net* net, const ppo_batch* b, const float* dlogits, const float* dvalues,
                               float* grad, void* ws, size_t ws_bytes, void* stream) {
  TuneScope tsc(net);
  if (!net || !b || !dlogits || !dvalues || !grad) return fail(PPO_EINVAL, "null argument");
  Sched S;
  const ppo_status st = schedule(net, b, S);
  if (st != PPO_OK) return st;
  const WsLayout w = plan(net, S.F, b->nb, true);
  if (const ppo_status fs = check_frames(net, S.F); fs != PPO_OK) return fs;
  if (!ws || ws_bytes < w.total) return fail(PPO_EWORKSPACE, "workspace needs %zu bytes", w.total);
  if (!al256(ws)) return fail(PPO_EWORKSPACE, "workspace must be 256-byte aligned");
  hipStream_t s = strm(stream);
  Ctx c{net, &w, (char*)ws, b->params, b->params_lp, grad, s, S.F};
  const ppo_net_desc& d = net->d;
  const float* feat = learner_fwd(c, b, S);  // activations recomputed here
  launch_head_bwd(dlogits, dvalues, S.F, d.hidden, d.num_actions, c.pf(net->head_w), c.at(w.dout),
                  c.at(w.dh0), s);
  learner_bwd(c, b, S, feat);
  return check_launch();
}

ppo_status ppo_policy_backward_ex(ppo_net* net, const ppo_batch* b, const float* dlogits, const float* dvalues,
                                  float* grad, float* dgoal, void* ws, size_t ws_bytes, void* stream) {
  TuneScope tsc(net);
  if (!net || !b || !dlogits || !dvalues || (!grad && !dgoal)) return fail(PPO_EINVAL, "null argument");
  if (dgoal && net->d.goal_mode != PPO_GOAL_VEC3) return fail(PPO_EINVAL, "a goal gradient needs PPO_GOAL_VEC3");
  Sched S;
  const ppo_status st = schedule(net, b, S);
  if (st != PPO_OK) return st;
  const WsLayout w = plan(net, S.F, b->nb, true);
  if (const ppo_status fs = check_frames(net, S.F); fs != PPO_OK) return fs;
  if (!ws || ws_bytes < w.total) return fail(PPO_EWORKSPACE, "workspace needs %zu bytes", w.total);
  if (!al256(ws)) return fail(PPO_EWORKSPACE, "workspace must be 256-byte aligned");
  hipStream_t s = strm(stream);
  Ctx c{net, &w, (char*)ws, b->params, b->params_lp, grad, s, S.F};
  const ppo_net_desc& d = net->d;
  const float* feat = learner_fwd(c, b, S);
  launch_head_bwd(dlogits, dvalues, S.F, d.hidden, d.num_actions, c.pf(net->head_w), c.at(w.dout),
                  c.at(w.dh0), s);
  learner_bwd(c, b, S, feat, dgoal);
  return check_launch();
}

ppo_status ppo_encode(ppo_net* net, const void* obs, int frames, const float* params, const void* params_lp,
                      float* feat, void* ws, size_t ws_bytes, void* stream) {
  TuneScope tsc(net);
  if (!net || !obs || !params || !feat || (net->prec && !params_lp)) return fail(PPO_EINVAL, "null argument");
  if (frames <= 0) return fail(PPO_ESHAPE, "frames must be positive");
  const WsLayout w = plan(net, frames, 1, false);
  if (const ppo_status fs = check_frames(net, frames); fs != PPO_OK) return fs;
  if (!ws || ws_bytes < w.total) return fail(PPO_EWORKSPACE, "workspace needs %zu bytes", w.total);
  if (!al256(ws)) return fail(PPO_EWORKSPACE, "workspace must be 256-byte aligned");
  hipStream_t s = strm(stream);
  Ctx c{net, &w, (char*)ws, params, params_lp, nullptr, s, frames};
  c.keep_u = false;
  const ppo_net_desc& d = net->d;
  launch_prep(obs, d.trunk == PPO_TRUNK_NONE ? 0 : net->prec, nullptr, frames, d.in_ch, d.in_hw, d.in_hw,
              d.avgpool, c.at(w.x0), s);
  const float* f = encoder_fwd(c);
  launch_copy2d(f, net->flat, frames, net->flat, feat, net->flat, s);
  return check_launch();
}

ppo_status ppo_planner_goal(const float* raw, int ld_raw, const int32_t* dst, int frames, float* goal,
                            void* stream) {
  if (!raw || !goal) return fail(PPO_EINVAL, "null argument");
  if (frames < 0 || ld_raw < 3) return fail(PPO_ESHAPE, "bad sizes");
  launch_planner_goal(raw, ld_raw, dst, frames, goal, strm(stream));
  return check_launch();
}

ppo_status ppo_planner_goal_backward(const float* raw, int ld_raw, const float* dgoal, int frames, float* draw,
                                     void* stream) {
  if (!raw || !dgoal || !draw) return fail(PPO_EINVAL, "null argument");
  if (frames < 0 || ld_raw < 3) return fail(PPO_ESHAPE, "bad sizes");
  launch_planner_goal_bwd(raw, ld_raw, dgoal, frames, draw, strm(stream));
  return check_launch();
}

ppo_status ppo_loss_head(ppo_net* net, const ppo_batch* b, const ppo_loss_cfg* cfg, const float* d_loss_scale,
                         const float* logits, const float* values, float* dlogits, float* dvalues, float* stats,
                         float* loss_out, void* ws, size_t ws_bytes, void* stream) {
  return loss_head(net, b, cfg, d_loss_scale, logits, values, dlogits, dvalues, stats, loss_out, ws, ws_bytes,
                   stream, false);
}

ppo_status ppo_loss_head_noalloc(ppo_net* net, const ppo_batch* b, const ppo_loss_cfg* cfg,
                                 const float* d_loss_scale, const float* logits, const float* values,
                                 float* dlogits, float* dvalues, float* stats, float* loss_out, void* stream) {
  void* p = nullptr;
  const ppo_status st = static_scratch(&p);
  if (st != PPO_OK) return st;
  return loss_head(net, b, cfg, d_loss_scale, logits, values, dlogits, dvalues, stats, loss_out, p,
                   sizeof(scratch), stream, true);
}

size_t ppo_loss_head_noalloc_max_frames(void) { return kNoAllocFrames; }

size_t ppo_adam_workspace_size(size_t P) {
  (void)P;
  return adam_ws_bytes();
}

ppo_status ppo_adam_step(float* master, const float* grad, float* m, float* v, void* lp_copy, size_t P,
                         const ppo_adam_cfg* cfg, ppo_scaler* scaler, void* ws, size_t ws_bytes,
                         void* stream) {
  if (!master || !grad || !m || !v || !cfg || !scaler) return fail(PPO_EINVAL, "null argument");
  if (P == 0) return fail(PPO_ESHAPE, "empty parameter vector");
  if (!ws || ws_bytes < adam_ws_bytes()) return fail(PPO_EWORKSPACE, "adam workspace too small");
  if (!(cfg->lr > 0.f) || !(cfg->beta1 >= 0.f && cfg->beta1 < 1.f) || !(cfg->beta2 >= 0.f && cfg->beta2 < 1.f) ||
      !(cfg->eps > 0.f))
    return fail(PPO_EINVAL, "bad Adam hyper-parameters");
  launch_adam(master, grad, m, v, (bf16_t*)lp_copy, P, cfg->lr, cfg->beta1, cfg->beta2, cfg->eps,
              cfg->growth_interval, scaler, ws, strm(stream));
  return check_launch();
}

ppo_status ppo_bench_unit_gemm(ppo_net* net, int op, int unit, int frames, const float* params,
                               const void* params_lp, float* grad, void* ws, size_t ws_bytes, int reps,
                               double* flops, void* stream) {
  TuneScope tsc(net);
  if (!net || !params || !grad || !flops || (net->prec && !params_lp)) return fail(PPO_EINVAL, "null argument");
  if (unit < 0 || unit >= (int)net->units.size() || op < 0 || op > 3 || frames <= 0 || reps <= 0)
    return fail(PPO_EINVAL, "bad unit / op / frames / reps");
  const WsLayout w = plan(net, frames, 1, true);
  if (const ppo_status fs = check_frames(net, frames); fs != PPO_OK) return fs;
  if (!ws || ws_bytes < w.total) return fail(PPO_EWORKSPACE, "workspace needs %zu bytes", w.total);
  if (!al256(ws)) return fail(PPO_EWORKSPACE, "workspace must be 256-byte aligned");
  hipStream_t s = strm(stream);
  Ctx c{net, &w, (char*)ws, params, params_lp, grad, s, frames};
  const Unit& u = net->units[unit];
  const ConvGeo g = geo(u, frames);
  const double M = (double)frames * u.Hout * u.Wout, N = u.Cout, K = (double)u.K * u.K * u.Cin / u.groups;
  *flops = 2.0 * M * N * K;
  // operands: scratch buffers sized for the largest unit of a learner call
  float *X = c.at(w.ga), *DY = c.at(w.gb), *OUT = c.at(w.gu);
  // op 3: the act step's product, its split-K partial tiles left for the GroupNorm
  const bool act_form = op == 3 && gn_one_launch(c, u);
  for (int r = 0; r < reps && u.groups > 1; ++r) {   // grouped: the direct convolution kernels
    if (op == 0 || op == 3) launch_gconv_fwd(net->prec, g, u.groups, X, c.wt(u.w), OUT, s);
    else if (op == 1) launch_gconv_dgrad(net->prec, g, u.groups, DY, c.wt(u.w), OUT, 0, s);
    else launch_gconv_wgrad(net->prec, g, u.groups, X, DY, grad + u.w, c.splitk(), kSplitKBytes, s);
  }
  Epi eact = epi(OUT, u.Cout);
  eact.act = act_form ? 1 : 0;
  if (act_form && act_fused_forms()) {   // the act step's group-major stores
    eact.gm_p = u.Hout * u.Wout;
    eact.gm_cg = u.Cout / net->d.gn_groups;
  }
  for (int r = 0; r < reps && u.groups == 1; ++r) {
    if (op == 0 || op == 3)
      gemm_conv_fwd(net->prec, g, X, c.wt(u.w), op == 3 ? eact : epi(OUT, u.Cout), kSplitKBytes, c.splitk(), s,
                    act_form);
    else if (op == 1)
      gemm_conv_dgrad(net->prec, g, DY, c.wt(u.w), c.at<void>(w.wT), epi(OUT, u.Cin), kSplitKBytes, c.splitk(), s);
    else
      gemm_conv_wgrad(net->prec, g, X, DY, epi(grad + u.w, u.K * u.K * u.Cin), kSplitKBytes, c.splitk(), s);
  }
  return check_launch();
}

ppo_status ppo_autotune(ppo_net* net, int mode, int* entries) {
  if (!net) return fail(PPO_EINVAL, "null argument");
  if (mode < -1 || mode > 1) return fail(PPO_EINVAL, "mode must be -1, 0 or 1");
  if (mode == -1) {
    net->tune.best.clear();
    net->tune.tuning = 0;
  } else {
    net->tune.tuning = mode;
  }
  if (entries) *entries = (int)net->tune.best.size();
  return PPO_OK;
}

ppo_status ppo_autotune_table(ppo_net* net, int write, int64_t* table, int capacity, int* entries) {
  if (!net || !entries || (capacity > 0 && !table) || capacity < 0) return fail(PPO_EINVAL, "bad arguments");
  if (write) {
    const int n = *entries;
    if (n < 0 || n > capacity) return fail(PPO_EINVAL, "entries outside the table");
    for (int i = 0; i < n; ++i) {
      const int64_t* r = table + 7 * i;
      if (r[5] < 0 || r[5] >= kGemmTiles || r[6] < 1 || r[6] > 256) return fail(PPO_EINVAL, "bad tile or split in row %d", i);
      net->tune.best[{r[0], r[1], r[2], r[3], r[4]}] = {(int)r[5], (int)r[6]};
    }
    *entries = (int)net->tune.best.size();
    return PPO_OK;
  }
  int i = 0;
  for (const auto& kv : net->tune.best) {
    if (i < capacity) {
      int64_t* r = table + 7 * i;
      for (int k = 0; k < 5; ++k) r[k] = kv.first[k];
      r[5] = kv.second.first;
      r[6] = kv.second.second;
    }
    ++i;
  }
  *entries = i;
  return PPO_OK;
}

ppo_status ppo_gemm_timer_arm(ppo_net* net, int unit, int op, int max_launches) {
  if (!net) return fail(PPO_EINVAL, "null argument");
  for (hipEvent_t e : net->timer_ev)
    if (e) (void)hipEventDestroy(e);
  net->timer_ev.clear();
  net->timer = GemmTimer{};
  net->timer_unit = net->timer_op = -1;
  if (unit < 0 && unit != PPO_TIMER_ALL_UNITS) return PPO_OK;
  if (unit >= (int)net->units.size() || op < 0 || op > 2 || max_launches <= 0 || max_launches > (1 << 16))
    return fail(PPO_EINVAL, "bad unit / op / max_launches");
  net->timer_ev.resize(2 * (size_t)max_launches);
  for (hipEvent_t& e : net->timer_ev)
    if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
      return fail(PPO_EDEVICE, "hipEventCreate failed");
    }
  net->timer = GemmTimer{net->timer_ev.data(), net->timer_ev.data() + max_launches, max_launches, 0, 0.0, 0.0};
  net->timer_unit = unit;
  net->timer_op = op;
  return PPO_OK;
}

ppo_status ppo_gemm_timer_read(ppo_net* net, int* launches, double* total_ms, double* flops, double* wbytes) {
  if (!net || !launches || !total_ms || !flops) return fail(PPO_EINVAL, "null argument");
  double t = 0.0;
  for (int i = 0; i < net->timer.n; ++i) {
    float ms = 0.f;
    if (hipEventSynchronize(net->timer.end[i]) != hipSuccess ||
        hipEventElapsedTime(&ms, net->timer.start[i], net->timer.end[i]) != hipSuccess)
      return fail(PPO_EDEVICE, "timer event query failed");
    t += ms;
  }
  *launches = net->timer.n;
  *total_ms = t;
  *flops = net->timer.flops;
  if (wbytes) *wbytes = net->timer.wbytes;
  net->timer.n = 0;
  net->timer.flops = 0.0;
  net->timer.wbytes = 0.0;
  return PPO_OK;
}

ppo_status ppo_workspace_probe(const ppo_net* net, int op, int max_frames, int max_envs, int kind,
                               int index, const char** name, int* relu, size_t* offset, int dims[4]) {
  if (!net || !offset || !dims) return fail(PPO_EINVAL, "null argument");
  if (max_frames <= 0 || max_envs <= 0 || max_envs > kMaxMbEnvs) return fail(PPO_ESHAPE, "bad sizes");
  const WsLayout w = plan(net, max_frames, max_envs, op == PPO_OP_LEARN);
  dims[0] = dims[1] = dims[2] = dims[3] = 0;
  if (name) *name = "";
  if (relu) *relu = 0;
  *offset = 0;
  if (kind == 0) {
    if (index < 0 || index >= (int)net->units.size()) return fail(PPO_EINVAL, "unit index out of range");
    const Unit& u = net->units[index];
    *offset = w.a[index];
    dims[0] = u.Hout;
    dims[1] = u.Wout;
    dims[2] = u.Cout;
    dims[3] = index == net->compress ? 1 : 0;
    if (name) *name = u.name.c_str();
    if (relu) *relu = u.relu;
    return PPO_OK;
  }
  if (kind == 1) {
    if (net->d.trunk == PPO_TRUNK_TINY) return fail(PPO_EINVAL, "no max pool in this trunk");
    *offset = w.arg;
    dims[0] = net->pool_h;
    dims[1] = net->pool_w;
    dims[2] = net->d.base_width;
    return PPO_OK;
  }
  if (kind == 2) {
    *offset = w.z;
    dims[0] = net->din0;
    dims[1] = net->d.vis_hidden;
    return PPO_OK;
  }
  if (kind == 3) {
    dims[0] = (int)net->units.size();
    return PPO_OK;
  }
  if (kind == 5) {
    if (net->d.trunk == PPO_TRUNK_TINY) return fail(PPO_EINVAL, "no max pool in this trunk");
    *offset = w.pool;
    dims[0] = net->pool_h;
    dims[1] = net->pool_w;
    dims[2] = net->d.base_width;
    return PPO_OK;
  }
  if (kind == 6 || kind == 7) {
    if (index < 0 || index >= net->d.lstm_layers) return fail(PPO_EINVAL, "layer index out of range");
    *offset = kind == 6 ? w.hp[index] : w.hout[index];
    dims[0] = net->d.hidden;
    return PPO_OK;
  }
  if (kind == 9) {
    if (op != PPO_OP_LEARN || index < 0 || index > 2)
      return fail(PPO_EINVAL, "benchmark operands: op PPO_OP_LEARN, index 0..2");
    *offset = index == 0 ? w.ga : index == 1 ? w.gb : w.gu;
    dims[0] = (int)std::min<size_t>((size_t)max_frames * net->max_unit, INT32_MAX);
    return PPO_OK;
  }
  if (kind == 8) {
    if (index < 0 || index >= (int)net->blocks.size() || net->blocks[index].R == 0)
      return fail(PPO_EINVAL, "block %d has no squeeze-excite gate", index);
    *offset = w.sea[index];
    dims[0] = net->blocks[index].R;
    dims[1] = net->units[net->blocks[index].c3].Cout;
    return PPO_OK;
  }
  if (kind == 4) {
    if (op != PPO_OP_LEARN) return fail(PPO_EINVAL, "the recurrence status is in learner workspaces");
    *offset = w.sync + lstm_error_word_offset();
    dims[0] = 1;
    return PPO_OK;
  }
  return fail(PPO_EINVAL, "unknown probe kind");
}

ppo_status ppo_cast_bf16(const float* src, void* dst, size_t n, void* stream) {
  if (!src || !dst) return fail(PPO_EINVAL, "null argument");
  if (n == 0) return PPO_OK;
  launch_cast_bf16(src, (bf16_t*)dst, n, strm(stream));
  return check_launch();
}

}  // extern "C"
