/*
 * ddppo.h -- C ABI of the MI355X (gfx950) hot path of one DD-PPO worker.
 *
 * Wijmans et al., "DD-PPO: Learning Near-Perfect PointGoal Navigators from
 * 2.5 Billion Frames", ICLR 2020.  One worker alternates an inference role
 * (batched act steps over its environments) and a learner role (GAE, the
 * clipped PPO objective of Eq. 2 and its gradient, then ParamUpdate of
 * Eq. 3-4).  On one worker the AllReduce of Eq. 3-4 is the identity, so the
 * gradient that ppo_loss_backward writes is what ppo_adam_step consumes.
 *
 * Conventions for every call:
 *   - Pointers named d_* or documented as "device" are device memory owned
 *     by the caller; "host" pointers are read before the call returns.  The
 *     compute calls allocate no device memory: scratch space is the caller's
 *     workspace (size from ppo_workspace_size).  The exceptions are
 *     benchmark and tuning aids, each documented below: a GEMM problem timed
 *     by the tile autotuner (ppo_autotune mode 1) allocates and frees a
 *     scratch output, and ppo_gemm_timer_arm creates HIP events.  With
 *     PPO_COLLECT_GRAPH, ppo_collect creates and keeps HIP graphs (the HIP
 *     runtime's memory) and one private capture stream per net.
 *   - All work is enqueued on `stream` (a hipStream_t passed as void*;
 *     NULL = the null stream) and is asynchronous.  Shape, pointer and
 *     workspace errors are detected on the host before any launch and
 *     return a negative ppo_status; a failed launch returns PPO_EDEVICE.
 *     Faults inside kernels surface at the caller's next synchronisation.
 *     No call aborts, exits or throws.  ppo_last_error() returns a
 *     thread-local message describing the last failure.
 *   - A ppo_net is a host-side descriptor.  It is not re-entrant across
 *     streams: calls that share one ppo_net must be ordered.
 *   - Environment switches (read at each call; for tests and measurement):
 *     DDPPO_GN_FUSED_MAX / DDPPO_GNB_FUSED_MAX (element count below which a
 *     GroupNorm forward / backward runs as one launch per image and group;
 *     4M / 1M), DDPPO_ACT_FUSED=0 (the act step's plain forms: convolution
 *     outputs stored NHWC, a separate max pool and projection-shortcut
 *     GroupNorm; the results are the same bit for bit), DDPPO_LSTM_SEQ=0 /
 *     DDPPO_LSTM_SEQ2=0 (the learner's recurrence one step per launch / one
 *     persistent launch per layer instead of both layers in one).
 *
 * Flat parameter format (float32 master, grads, Adam moments; the bfloat16
 * working copy has the same order).  Tensors in order:
 *   tiny trunk  : conv1 [c1][3][3][in_ch], gn1 gamma [c1], beta [c1],
 *                 conv2 [c2][3][3][c1],  gn2 gamma [c2], beta [c2]
 *   resnet trunk: stem [w0][7][7][in_ch], gamma, beta [w0]; per stage s (width
 *                 w = w0*2^s) and block j: c1 [w][1][1][cin] + gn, c2 [w][3][3][w]
 *                 + gn, c3 [4w][1][1][w] + gn, and on block 0 a projection
 *                 ds [4w][1][1][cin] + gn; compress [cc][3][3][32*w0] + gn
 *                 (every "+ gn" is gamma then beta, one value per output channel)
 *   visual FC   : W [vis_hidden][flat] with input index (channel, row, col), b
 *   goal FC     : W [goal_dim][3], b            (goal_mode = polar only)
 *   embedding   : E [num_actions+1][prev_act_dim] (prev_act_dim > 0 only;
 *                 row 0 is the start token)
 *   LSTM layer l: W [4H][in_l + H] (input columns then recurrent columns,
 *                 gate row blocks i, f, g, o), b [4H]
 *   heads       : W [num_actions+1][H] (policy rows, then the value row), b
 * Convolution weights are (out, kh, kw, in).  Convolutions have no bias.
 *
 * Rollout arrays are time-major: [T+1][N] for per-act-step data (step T is
 * the bootstrap step), [T][N] for per-transition data, frames
 * [T+1][N][C][H][W] (float32 or bfloat16 per the net's dtype).
 */
#ifndef DDPPO_H
#define DDPPO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PPO_OK = 0,
  PPO_EINVAL = -1,       /* null pointer, bad scalar argument */
  PPO_ESHAPE = -2,       /* inconsistent or unsupported sizes */
  PPO_EUNSUPPORTED = -3, /* feature or device not supported (non-gfx950) */
  PPO_EWORKSPACE = -4,   /* workspace too small or misaligned */
  PPO_EDEVICE = -5       /* a HIP call or launch failed */
} ppo_status;

enum { PPO_F32 = 0, PPO_BF16 = 1 };
enum { PPO_TRUNK_TINY = 0, PPO_TRUNK_RESNET = 1, PPO_TRUNK_SERESNEXT = 2, PPO_TRUNK_NONE = 3 };
enum { PPO_GOAL_RAW = 0, PPO_GOAL_POLAR = 1, PPO_GOAL_VEC3 = 2, PPO_GOAL_NONE = 3 };
enum { PPO_OP_ACT = 0, PPO_OP_LEARN = 1, PPO_OP_LOSS = 2 };

/* Network shape (appendix "Agent Design"; Sec. 4 "Agent").  The visual
 * encoder is the tiny two-conv trunk, or ResNet50 or SE-ResNeXt50 (Sec. 6,
 * Table 1) with every width halved and GroupNorm.  An SE-ResNeXt bottleneck
 * of stage s (w = base_width 2^s) is: 1x1 conv to 2w, 3x3 conv in
 * `cardinality` groups (stride on the first block of stages 1-3), 1x1 conv to
 * 4w, each with GroupNorm (and ReLU but the last), then a squeeze-excite gate
 * s = sigmoid(W2 relu(W1 mean_pixels(y) + b1) + b2) with W1 [4w/r][4w],
 * scaling the branch per channel before the shortcut is added and the ReLU;
 * its parameters follow the third convolution's in the flat format (se1.w,
 * se1.b, se2.w, se2.b). */
typedef struct ppo_net_desc {
  int in_ch;          /* frame channels (4: RGB-D)                              */
  int in_hw;          /* frame height = width (256)                             */
  int avgpool;        /* 1: 2x2 average pool before the trunk                   */
  int trunk;          /* PPO_TRUNK_TINY | _RESNET | _SERESNEXT | _NONE (features in:
                         frames are float32 [in_ch] vectors; in_hw 1, no avgpool)   */
  int tiny_ch[2];     /* tiny trunk widths (16, 32)                             */
  int base_width;     /* resnet stem width; stage widths w0*2^s (32)            */
  int blocks[4];      /* bottlenecks per stage (3, 4, 6, 3)                     */
  int gn_groups;      /* GroupNorm groups (16 resnet, 8 tiny)                   */
  int compress_ch;    /* compression conv output channels (128)                 */
  int vis_hidden;     /* visual FC width (512)                                  */
  int goal_mode;      /* PPO_GOAL_RAW: [2] concatenated; PPO_GOAL_POLAR: (d, theta)
                         -> [d, cos, sin] -> FC; PPO_GOAL_VEC3: a given [3] -> FC;
                         PPO_GOAL_NONE: no goal input (goal_dim 0, goal may be NULL) */
  int goal_dim;       /* 2 for raw, FC width for polar                          */
  int prev_act_dim;   /* previous-action embedding width, 0 = none              */
  int lstm_layers;    /* 1 or 2                                                 */
  int hidden;         /* LSTM hidden size (512)                                 */
  int num_actions;    /* 4                                                      */
  int dtype;          /* PPO_F32 | PPO_BF16: GEMM operand precision             */
  int cardinality;    /* seresnext: groups of each bottleneck's 3x3 convolution (16) */
  int se_reduction;   /* seresnext: squeeze-excite hidden width = C / se_reduction (16) */
  int prev_actions;   /* previous-action vocabulary of the embedding (0: num_actions);
                         the table has prev_actions + 1 rows (start token first)   */
} ppo_net_desc;

typedef struct ppo_net ppo_net;

/* Validate a description and build the host-side plan.  No device memory is
 * allocated.  Errors: PPO_EINVAL (null), PPO_ESHAPE (sizes that do not
 * divide: e.g. widths not multiples of gn_groups, a trunk that does not
 * reduce in_hw to an integer map), PPO_EUNSUPPORTED (the current HIP device
 * is not a gfx950), PPO_EDEVICE (the device cannot be queried).  With no
 * HIP device visible the plan is still built (sizes and offsets can be
 * read); compute calls then fail with PPO_EDEVICE. */
ppo_status ppo_net_create(const ppo_net_desc* desc, ppo_net** out);
void ppo_net_destroy(ppo_net* net);

/* Number of float parameters in the flat format above. */
size_t ppo_param_count(const ppo_net* net);

/* Offset and element count of the i-th tensor of the flat format, with its
 * name (static string).  Returns PPO_EINVAL past the last tensor. */
ppo_status ppo_param_tensor(const ppo_net* net, int i, const char** name, size_t* offset,
                            size_t* count);

/* Workspace bytes for one call of ppo_act (op = PPO_OP_ACT, max_frames = the
 * largest act batch), ppo_loss_backward / ppo_policy_forward /
 * ppo_policy_backward (op = PPO_OP_LEARN, max_frames = the largest number of
 * valid frames of one minibatch, max_envs its env count) or ppo_loss_head
 * (op = PPO_OP_LOSS, same sizes; a few bytes per frame).  The workspace must
 * be 256-byte aligned device memory. */
ppo_status ppo_workspace_size(const ppo_net* net, int op, int max_frames, int max_envs,
                              size_t* bytes);

/* ---------------------------------------------------------------------------
 * ppo_act -- one batched act step of the inference role (Sec. 3, Sec. 4).
 * For each of `batch` envs b: frame -> encoder -> [visual FC | goal | prev-action
 * embedding] -> LSTM (h, c first multiplied by mask[b]; mask 0 also selects
 * the start token) -> logits, value; action = the smallest k whose cumulative
 * softmax probability exceeds u[b] (the last action if rounding leaves none),
 * logp = log pi(action).
 *
 * `active` (device int32, or NULL = all rows) serves rollouts whose envs stop
 * at different steps (preemption, Sec. 3) from one captured graph: every row
 * is computed, but action, logp, value, logits, h_out and c_out are written
 * only for rows b < *active, read on the device when the kernels run (so the
 * host may change it between replays); rows >= *active keep their previous
 * contents (with h_out aliasing h_in, their state).  Values outside
 * [0, batch] act as the nearer bound.  Rows are independent, so rows
 * b < *active are bit-for-bit those of a call without the count.
 */
typedef struct ppo_act_io {
  int batch;                  /* B envs (rows) in this call                     */
  int state_rows;             /* rows per layer of h/c arrays (>= batch; 0 = batch) */
  const void* obs;            /* device [B][C][H][W], float32 or bfloat16       */
  const float* goal;          /* device [B][2]: (d, theta) or the raw 2-vector   */
  const int32_t* prev_action; /* device [B] action taken at the previous step   */
  const float* mask;          /* device [B]: 0 at an episode start, else 1      */
  const float* h_in;          /* device [L][state_rows][H], rows < B are read    */
  const float* c_in;          /* device [L][state_rows][H]                      */
  const float* u;             /* device [B] uniforms in [0,1)                   */
  const float* params;        /* device flat float32 parameters                 */
  const void* params_lp;      /* device flat bfloat16 copy (PPO_BF16), else NULL */
  int32_t* action;            /* device [B] out                                 */
  float* logp;                /* device [B] out                                 */
  float* value;               /* device [B] out                                 */
  float* h_out;               /* device [L][state_rows][H] out, rows < B (may alias h_in) */
  float* c_out;               /* device [L][state_rows][H] out (may alias c_in) */
  float* logits;              /* device [B][A] out, or NULL                     */
  const int32_t* active;      /* device [1] rows written (see above), or NULL   */
} ppo_act_io;

ppo_status ppo_act(ppo_net* net, const ppo_act_io* io, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * ppo_collect -- the rollout's T+1 dependent act steps (Sec. 3 "inference":
 * T = 128 steps of experience, plus the step that gives the bootstrap value
 * V(s_T)), each one ppo_act over the rollout's buffers:
 *
 *   step t reads    obs[t], goal[t], mask[t], u[t], actions[t] (previous
 *                   action), h_hist[t], c_hist[t];
 *   step t writes   actions[t+1], logp[t], value[t], and its next state to
 *                   h_hist[t+1], c_hist[t+1] (to h_last, c_last at t = T).
 *
 * Only steps t_begin <= t < t_end run (the full rollout: 0, T+1), so a
 * caller that decides after each step whether the rollout ends (preemption,
 * Sec. 3) runs one step per call.
 *
 * Rows: with `active` (device int32 [T+1], or NULL = all N) step t writes
 * rows b < active[t] only, read on the device when the step runs (ppo_act's
 * row count).  With PPO_COLLECT_TRIM, `lengths` (host int32 [N], T_n,
 * non-increasing: envs ordered longest first) instead launches step t on
 * its rows b with T_b >= t only, and the steps stop at the first step with
 * none; `active` is then ignored.
 *
 * PPO_COLLECT_GRAPH: the steps run as a HIP graph the library captures and
 * owns, one per distinct argument set (every field below, ws, ws_bytes, the
 * flags and, with PPO_COLLECT_TRIM, the contents of `lengths`).  The first
 * call with a new argument set runs the steps eagerly on `stream` (so the
 * tile table is tuned when tuning is on; the results are that call's
 * outputs) and then records them, on a private stream of the net's device,
 * into a graph that later calls launch on `stream`.  A graph reads the
 * buffers' contents when it runs, not when it was captured, so the host may
 * refill obs, u, active, ... between launches; the buffers themselves must
 * stay allocated while a graph keyed on them may still be launched.  At
 * most 1024 graphs are kept per net (the oldest is dropped, after the device
 * is idle); ppo_collect_clear drops them all.  When `stream` is itself
 * being captured, the steps are recorded into the caller's graph as plain
 * launches.
 *
 * Errors (null pointer, bad step range, unordered lengths, small workspace)
 * are reported before any launch.  A graph that cannot be captured or
 * instantiated gives PPO_EDEVICE; the eager results of that call stand.
 */
enum { PPO_COLLECT_GRAPH = 1, PPO_COLLECT_TRIM = 2 };

typedef struct ppo_collect_io {
  int T;                      /* rollout steps: act steps 0..T                  */
  int N;                      /* envs (rows of every [..][N] array)             */
  int t_begin, t_end;         /* steps run by this call, 0 <= t_begin <= t_end <= T+1 */
  const void* obs;            /* device [T+1][N][C][H][W] (bfloat16 on a PPO_BF16 net
                                 with a visual trunk, float32 otherwise)         */
  const float* goal;          /* device [T+1][N][goal width], NULL for PPO_GOAL_NONE */
  const float* mask;          /* device [T+1][N]                                 */
  const float* u;             /* device [T+1][N] uniforms in [0,1)               */
  const int32_t* active;      /* device [T+1] rows written per step, or NULL     */
  const int32_t* lengths;     /* host [N] T_n (PPO_COLLECT_TRIM only), or NULL = all T */
  const float* params;        /* device flat float32 parameters                  */
  const void* params_lp;      /* device flat bfloat16 copy (PPO_BF16), else NULL  */
  int32_t* actions;           /* device [T+2][N]: row 0 the action before step 0
                                 (read), row t+1 step t's action (written)       */
  float* logp;                /* device [T+1][N] out                             */
  float* value;               /* device [T+1][N] out                             */
  float* h_hist;              /* device [T+1][L][N][H]: row 0 read, rows 1..T written */
  float* c_hist;              /* device [T+1][L][N][H]                           */
  float* h_last;              /* device [L][N][H]: state written by step T       */
  float* c_last;              /* device [L][N][H]                                */
} ppo_collect_io;

/* ws: ppo_act's workspace for max_frames = N.  stream: the caller's. */
ppo_status ppo_collect(ppo_net* net, const ppo_collect_io* io, int flags, void* ws, size_t ws_bytes,
                       void* stream);

/* Drops every graph ppo_collect keeps for this net (after the device is
 * idle); returns how many were dropped.  Call it before freeing buffers
 * that a kept graph is keyed on if their addresses may be reused with other
 * shapes, or to release the graphs' memory. */
int ppo_collect_clear(ppo_net* net);

/* Number of graphs ppo_collect keeps for this net. */
int ppo_collect_graph_count(const ppo_net* net);

/* ---------------------------------------------------------------------------
 * ppo_gae -- generalized advantage estimation (Sec. 4 "Training": gamma, GAE
 * parameter tau = lambda).  For each env n, t = len[n]-1 .. 0 with A = 0 past
 * the end:  delta_t = r_t + gamma (1-d_t) V_{t+1} - V_t,
 *           A_t = delta_t + gamma lambda (1-d_t) A_{t+1},  R_t = A_t + V_t.
 * A rollout cut at len[n] < T (preemption, Sec. 3) bootstraps with V[len[n]].
 * rew, done [T][N]; val [T+1][N]; len [N] device int32 or NULL (all T).
 * adv, ret [T][N] float32 out (0 past len).  adv_stats: device double[2]
 * (population mean and variance of the valid advantages, float64) or NULL.
 */
ppo_status ppo_gae(const float* rew, const float* val, const uint8_t* done, const int32_t* len,
                   int T, int N, float gamma, float lambda, float* adv, float* ret,
                   double* adv_stats, void* stream);

/* ---------------------------------------------------------------------------
 * ppo_loss_backward -- learner forward and backward for one minibatch of
 * whole env sequences (Sec. 3-4).  Re-runs the policy over every frame
 * t < T_n of the chosen envs from the stored rollout-start state, then
 *   L = -sum_n w_n sum_t min(r A, clip(r, 1-eps, 1+eps) A)          (Eq. 2)
 *       + c_v sum_n w_n sum_t 1/2 (V - R)^2 - c_e sum_n w_n sum_t H(pi),
 *   r = exp(logp - logp_old), w_n = 1/(|B| T_n) (every env weighs equally, Sec. 3)
 * and writes grad = S * dL/dtheta (S = *d_loss_scale, 1 for float32 nets).
 */
typedef struct ppo_batch {
  int T;                      /* rollout steps (row count of [T][N] arrays)      */
  int N;                      /* envs in the rollout (row length)               */
  int nb;                     /* envs in this minibatch                          */
  const int32_t* env_ids;     /* host [nb] env indices                           */
  const int32_t* lengths;     /* host [N] T_n (1..T), or NULL for all T          */
  const void* obs;            /* device [T+1][N][C][H][W]                        */
  const float* goal;          /* device [T+1][N][2]                              */
  const int32_t* prev_action; /* device [T+1][N] prev-action input of each step  */
  const float* mask;          /* device [T+1][N] episode mask of each step       */
  const int32_t* action;      /* device [T+1][N] actions taken                   */
  const float* logp_old;      /* device [T+1][N]                                 */
  const float* adv;           /* device [T][N]                                   */
  const float* ret;           /* device [T][N]                                   */
  const float* h0;            /* device [L][N][H] state at the rollout start     */
  const float* c0;            /* device [L][N][H]                                */
  const float* params;        /* device flat float32                             */
  const void* params_lp;      /* device flat bfloat16 copy, or NULL (PPO_F32)    */
} ppo_batch;

typedef struct ppo_loss_cfg {
  float clip;                 /* epsilon of Eq. 2 (0.2)                          */
  float value_coef;           /* c_v (0.5)                                       */
  float entropy_coef;         /* c_e (0.01)                                      */
  int norm_adv;               /* 1: A <- (A - mean)/(std + 1e-5) (off in the paper) */
  const double* adv_stats;    /* device double[2] from ppo_gae when norm_adv     */
} ppo_loss_cfg;

/* stats (device float[8]): loss, policy term, value term, entropy term,
 * clip fraction, approximate KL, min ratio, max ratio (weighted like L). */
ppo_status ppo_loss_backward(ppo_net* net, const ppo_batch* b, const ppo_loss_cfg* cfg,
                             const float* d_loss_scale, float* grad, float* stats, void* ws,
                             size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * The learner split in two, for callers that form their own loss on the
 * policy outputs (e.g. an autograd function).  Both use the minibatch of
 * ppo_batch; the action/logp_old/adv/ret fields are not read.
 *
 * ppo_policy_forward: logits [F][A] and values [F] of every valid frame of
 * the minibatch (F = sum of the chosen envs' lengths), frames in the packed
 * order (time-major; envs sorted by length, longest first, ties in the given
 * order); frame_src [F] (device int32, or NULL) receives t*N + env of each
 * frame.  Nothing is kept in the workspace between calls.
 *
 * ppo_policy_backward: recomputes the same forward (activations are not
 * stored between the calls), then writes grad = d(sum dlogits*logits +
 * dvalues*values)/dtheta for the given dlogits [F][A], dvalues [F] in that
 * frame order.  Workspace sizes as for ppo_loss_backward.
 */
ppo_status ppo_policy_forward(ppo_net* net, const ppo_batch* b, float* logits, float* values,
                              int32_t* frame_src, void* ws, size_t ws_bytes, void* stream);
ppo_status ppo_policy_backward(ppo_net* net, const ppo_batch* b, const float* dlogits,
                               const float* dvalues, float* grad, void* ws, size_t ws_bytes,
                               void* stream);

/* ppo_policy_backward_ex -- ppo_policy_backward for nets used inside a larger
 * differentiable system (the neural controller of Sec. 6 "Transfer
 * Learning": a planner trained through a frozen controller).  grad may be
 * NULL: then no parameter gradient is formed (a frozen net) and only data
 * gradients run.  dgoal (PPO_GOAL_VEC3 nets, or NULL) receives the gradient
 * with respect to the goal input, [F][3] float32 in the packed frame order of
 * ppo_policy_forward.  At least one of grad and dgoal must be given. */
ppo_status ppo_policy_backward_ex(ppo_net* net, const ppo_batch* b, const float* dlogits,
                                  const float* dvalues, float* grad, float* dgoal, void* ws,
                                  size_t ws_bytes, void* stream);

/* ppo_encode -- the visual encoder alone (App. "Agent Design": average pool,
 * trunk, compression conv) on `frames` frames obs [frames][C][H][W] (float32,
 * or bfloat16 for PPO_BF16 nets): feat [frames][flat] float32 (channel, row,
 * column order: the visual FC's input).  No gradient, nothing kept.  The
 * workspace is that of ppo_act (op PPO_OP_ACT, max_frames >= frames).  Used
 * for a frozen encoder shared by several heads (the neural controller). */
ppo_status ppo_encode(ppo_net* net, const void* obs, int frames, const float* params, const void* params_lp,
                      float* feat, void* ws, size_t ws_bytes, void* stream);

/* ppo_planner_goal -- the neural controller's PointGoal (appendix "Neural
 * controller additional details") from the planner's raw head outputs:
 * goal = [ELU(r0) + 0.75, tanh(r1), tanh(r2)] (the direction is not
 * renormalised).  raw: row f at raw + f*ld_raw (the first 3 columns);
 * goal row dst[f] (device int32, or NULL for f) of a [*][3] float32 array.
 * ppo_planner_goal_backward: draw (rows of stride ld_raw, first 3 columns)
 * = dgoal [frames][3] (dense, row f) times the transform's derivative at raw
 * (ELU' = 1 for r > 0, exp(r) otherwise; tanh' = 1 - tanh^2). */
ppo_status ppo_planner_goal(const float* raw, int ld_raw, const int32_t* dst, int frames, float* goal,
                            void* stream);
ppo_status ppo_planner_goal_backward(const float* raw, int ld_raw, const float* dgoal, int frames, float* draw,
                                     void* stream);

/* ppo_loss_head -- the objective of ppo_loss_backward (Eq. 2 with the value
 * and entropy terms, weights w_n = 1/(|B| T_n) of Sec. 3, optional advantage
 * normalisation) evaluated on given policy outputs: logits [F][A] and values
 * [F] (device float32) of the minibatch's valid frames in the order of
 * ppo_policy_forward.  Writes stats [8] (as ppo_loss_backward), loss_out
 * [1] = S*L (device float32, or NULL) and the gradient of S*L with respect
 * to the outputs: dlogits [F][A], dvalues [F] (device float32; S =
 * *d_loss_scale for PPO_BF16 nets, 1 for PPO_F32).
 * Reads the minibatch's env_ids, lengths, mask, action, logp_old, adv and
 * ret fields only.  Workspace: ppo_workspace_size(op = PPO_OP_LOSS).  With
 * ppo_policy_forward / ppo_policy_backward it splits ppo_loss_backward in
 * three (a caller's autograd graph in between). */
ppo_status ppo_loss_head(ppo_net* net, const ppo_batch* b, const ppo_loss_cfg* cfg, const float* d_loss_scale,
                         const float* logits, const float* values, float* dlogits, float* dvalues, float* stats,
                         float* loss_out, void* ws, size_t ws_bytes, void* stream);

/* ppo_loss_head_noalloc -- ppo_loss_head without a workspace argument, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation).  Same arguments,
 * outputs and errors as ppo_loss_head; its scratch (frame map and per-frame
 * loss terms) is a static device array of the library, about 1.5 MB, held on
 * every GPU the library runs on until the process ends.  Allocates nothing,
 * on the device or the host.  Returns PPO_ESHAPE for a minibatch of more
 * valid frames than ppo_loss_head_noalloc_max_frames() (32768).  Every call
 * on one GPU uses that GPU's array: calls that overlap on one GPU (other
 * streams, other threads) race and must be ordered by the caller.  Nothing in
 * the array needs to start at zero (each call writes what it reads). */
ppo_status ppo_loss_head_noalloc(ppo_net* net, const ppo_batch* b, const ppo_loss_cfg* cfg,
                                 const float* d_loss_scale, const float* logits, const float* values,
                                 float* dlogits, float* dvalues, float* stats, float* loss_out, void* stream);
size_t ppo_loss_head_noalloc_max_frames(void);

/* ---------------------------------------------------------------------------
 * ppo_adam_step -- ParamUpdate of Eq. 3-4 (Adam, Kingma & Ba, with bias
 * correction; the paper's optimiser, Sec. 4 "Training").  Device state:
 *   scaler->scale S: gradients arrive multiplied by S and are unscaled here;
 *   if any unscaled gradient is not finite the step is skipped (params, m, v,
 *   step unchanged), S halves (only when growth_interval > 0) and skipped
 *   increments; otherwise step += 1,
 *     m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 *     theta -= lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps),
 *   and after `growth_interval` consecutive good steps S doubles (dynamic
 *   loss scaling; growth_interval 0 keeps S fixed, also on a skipped step).
 * master, m, v [P] float32 in place; grad [P] float32 (read only); lp_copy
 * [P] bfloat16 rewritten from the new master (NULL to skip).  ws: at least
 * ppo_adam_workspace_size(P) bytes of device scratch.
 */
typedef struct ppo_adam_cfg {
  float lr, beta1, beta2, eps;
  int growth_interval;        /* 2000 for bfloat16 nets, 0 for float32           */
} ppo_adam_cfg;

typedef struct ppo_scaler {   /* device-resident; initialise scale = 65536 or 1  */
  float scale;
  int32_t step;               /* Adam step count k (completed steps)             */
  int32_t good_steps;         /* consecutive finite steps since the last change  */
  int32_t skipped;            /* total skipped steps                             */
  int32_t found_inf;          /* last call: 1 if skipped                         */
  int32_t pad[3];
} ppo_scaler;

size_t ppo_adam_workspace_size(size_t P);

ppo_status ppo_adam_step(float* master, const float* grad, float* m, float* v, void* lp_copy,
                         size_t P, const ppo_adam_cfg* cfg, ppo_scaler* scaler, void* ws,
                         size_t ws_bytes, void* stream);

/* Test introspection of a workspace laid out for (op, max_frames, max_envs):
 * where a call leaves the forward activations that decided each ReLU, max
 * pool and bfloat16 operand rounding, so a reference implementation can take
 * the same decisions.  Frames are in the
 * call's packed order (time-major; envs sorted by length, longest first,
 * ties in the given order).
 *   kind 0: normalised output of trunk unit `index` (conv + GroupNorm [+ residual]
 *           [+ ReLU]) as float32; dims = {Ho, Wo, C, channel_major}
 *           (channel_major 1: [F][C][Ho*Wo], else [F][Ho][Wo][C]); *name = the
 *           unit's convolution tensor name; *relu = 1 if a ReLU produced it
 *   kind 1: max-pool winner (uint8 kh*3+kw) [F][h][w][C]; dims = {h, w, C, 0}
 *   kind 2: LSTM layer-0 input rows float32 [F][din0], columns < vis_hidden
 *           being the post-ReLU visual FC output; dims = {din0, vis_hidden, 0, 0}
 *   kind 3: dims[0] = number of trunk units
 *   kind 5: max-pool output float32 [F][h][w][C]; dims = {h, w, C, 0}
 *   kind 6: LSTM layer `index`'s masked previous state m_t h_{t-1}, float32
 *           [F][H] (the recurrent operand of the gate products); dims = {H, ..}
 *   kind 7: LSTM layer `index`'s output h_t, float32 [F][H]; dims = {H, ..}
 *   kind 8: squeeze-excite gate of bottleneck block `index` (SE-ResNeXt):
 *           its hidden pre-activation W1 z + b1, float32 [F][R]; dims = {R, C, 0, 0}
 *   kind 9 (op PPO_OP_LEARN): the operand buffers of ppo_bench_unit_gemm,
 *           float32 NHWC: index 0 the unit's input, 1 the gradient at its
 *           output, 2 the output written (forward / data gradient);
 *           dims[0] = floats each holds
 *   kind 4 (op PPO_OP_LEARN): the learner's recurrence status, one uint32;
 *           nonzero after a call means a device-wide barrier of the persistent
 *           LSTM launches gave up waiting (bounded wait) and the call's
 *           outputs were poisoned with NaN; cleared at the start of every
 *           learner call; dims = {1, 0, 0, 0}
 * Returns PPO_EINVAL for an index or kind that does not exist. */
ppo_status ppo_workspace_probe(const ppo_net* net, int op, int max_frames, int max_envs, int kind,
                               int index, const char** name, int* relu, size_t* offset, int dims[4]);

/* Benchmark aid: enqueue `reps` launches of the convolution GEMM of trunk
 * unit `unit` (op 0 forward, 1 data gradient, 2 weight gradient, as
 * ppo_loss_backward runs them; op 3 the forward product as ppo_act runs it at
 * this frame count, its split-K partial tiles left for the GroupNorm) at
 * `frames` frames, with the tile shape and K split of that call, on
 * workspace scratch data (workspace laid out as for ppo_loss_backward with
 * max_frames = frames, max_envs = 1).  *flops = 2*M*N*K of one launch.  The
 * weight-gradient op writes that unit's slot of grad. */
ppo_status ppo_bench_unit_gemm(ppo_net* net, int op, int unit, int frames, const float* params,
                               const void* params_lp, float* grad, void* ws, size_t ws_bytes, int reps,
                               double* flops, void* stream);

/* GEMM tile autotuner of this net.  mode 1: from now on, every GEMM problem
 * (operand kind, M, N, K, precision) that a call on this net meets and that
 * is not yet in the net's table is timed over the candidate tile shapes
 * (128x128 ... 32x128) and K splits before it runs; the call then
 * waits for those timings (so tune in warm-up, never under stream capture,
 * where tuning is skipped) and allocates a scratch output for them.  mode 0:
 * stop tuning, keep using the table.  mode -1: clear the table (heuristic
 * choice).  A product whose split-K partial tiles a GroupNorm sums is tuned
 * on a key of its own, timed with an ordered reduction standing in for the
 * GroupNorm's sum.  *entries (optional) = problems in the table.  Not thread-safe with other
 * calls on the same net. */
ppo_status ppo_autotune(ppo_net* net, int mode, int* entries);

/* The autotuner's table as rows of 7 int64: the problem key (operand kind,
 * M, N, K, precision/variant code) then the tile index (0..5: 128x128,
 * 128x64, 64x128, 64x64, 128x32, 32x128) and the K split.  write 0: copy up
 * to `capacity` rows into `table`, *entries = rows in the table (call with
 * capacity 0 for the count).  write 1: add or replace the first *entries rows
 * of `table` (e.g. a table read back from an earlier run, so that a profiled
 * run uses the same tiles); *entries = rows in the table afterwards.
 * Errors: PPO_EINVAL for a tile or split out of range. */
ppo_status ppo_autotune_table(ppo_net* net, int write, int64_t* table, int capacity, int* entries);

/* Benchmark aid: time the GEMM kernel launches of trunk unit `unit`
 * (PPO_TIMER_ALL_UNITS: every unit), op (0 forward, 1 data gradient, 2 weight
 * gradient) inside later library calls on this net, e.g. ppo_act or
 * ppo_loss_backward.  Events are recorded on the call's stream around each
 * GEMM kernel itself (a split-K reduction that follows it is not included),
 * for at most max_launches launches, never inside stream capture.  unit = -1
 * disarms and frees the events.  Creates HIP events; not thread-safe with
 * other calls on the same net. */
enum { PPO_TIMER_ALL_UNITS = -2 };
ppo_status ppo_gemm_timer_arm(ppo_net* net, int unit, int op, int max_launches);
/* Waits for the recorded launches and returns their count, summed duration
 * (ms), summed 2*M*N*K and (wbytes, or NULL) summed bytes of the weight
 * operands of the timed convolution forward products; then starts a new
 * count (still armed). */
ppo_status ppo_gemm_timer_read(ppo_net* net, int* launches, double* total_ms, double* flops, double* wbytes);

/* dst[i] = bfloat16(src[i]) (round to nearest even) for the initial working
 * copy of the parameters; later copies come from ppo_adam_step.  src [n]
 * float32, dst [n] bfloat16, both device. */
ppo_status ppo_cast_bf16(const float* src, void* dst, size_t n, void* stream);

const char* ppo_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DDPPO_H */
