/*
 * wsx.h -- C ABI of the GPU-resident roll-out library (libwsx.so, gfx950).
 *
 * The library runs the data-parallel hot path of a GPU-resident RL
 * workflow (arXiv 2408.00930, Sec. 2 and App. B): every environment replica
 * steps in place on the GPU, its agents sample actions from a policy model in
 * device memory, and the roll-out data are written to device memory for
 * training; discounted returns and GAE advantages (Sec. 3, actor-critic)
 * follow on the device. No call on the hot path copies data between host and
 * device.
 *
 * Conventions for every entry point:
 *  - Device buffers are owned by the caller (e.g. torch tensors) and passed as
 *    raw device pointers; the library never allocates device memory except
 *    where an entry point says so. Host pointers are read during the call only.
 *  - `stream` is a hipStream_t (NULL = the null stream). Work is enqueued
 *    asynchronously on it; no entry point synchronises the device unless it
 *    says so.
 *  - Return value: WSX_OK (0) or a negative error code. All arguments are
 *    validated on the host before anything is enqueued; on error nothing is
 *    enqueued and wsx_last_error() describes the failure (thread-local string,
 *    valid until the next call on that thread). No C++ exception crosses the
 *    ABI.
 *  - Layouts are row-major. "rows" are agents: one per environment for the
 *    single-agent kinds, the sum of agent counts for the market.
 */
#ifndef WSX_H
#define WSX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WSX_OK 0
#define WSX_EINVAL (-1)        /* invalid argument                                */
#define WSX_EUNSUPPORTED (-2)  /* valid but not supported (shape, dtype, kind)     */
#define WSX_EHIP (-3)          /* the HIP runtime reported an error                */
#define WSX_ESTATE (-4)        /* object used in a state that does not allow it    */
#define WSX_ETIMEOUT (-5)      /* a wait ended before the request completed        */
#define WSX_ECANCELED (-6)     /* the request was cancelled                        */

/* Environment kinds (App. C example families; dynamics are the project's
 * readings, see the design notes). */
#define WSX_CARTPOLE 1   /* state 4, obs 4, 2 discrete actions                   */
#define WSX_PENDULUM 2   /* state 2, obs 3, 1 continuous action (torque)         */
#define WSX_ACROBOT 3    /* state 4, obs 6, 1 continuous action (elbow torque)   */
#define WSX_MARKET 4     /* per agent: state 32, obs 32, 50 discrete actions      */
#define WSX_REACTION 5   /* state 21 (x[20], cached noisy energy), obs 20, 40 actions */

/* Element types. */
#define WSX_F32 0
#define WSX_BF16 1
#define WSX_FP8_E4M3 2   /* OCP E4M3FN                                           */
#define WSX_F64 3

/* Roll-out execution modes. */
#define WSX_MODE_FUSED 0   /* one persistent kernel for the whole horizon          */
#define WSX_MODE_PLAIN 1   /* per step: policy, sample and step kernels           */
#define WSX_MODE_GRAPH 2   /* the PLAIN launches captured once in a hipGraph and   */
                           /* replayed                                            */
#define WSX_MODE_FUSED_GRAPH 3 /* the horizon as persistent fused kernels of      */
                           /* chunk_steps steps each (wsx_env_set_chunk), captured */
                           /* once in a hipGraph and replayed                     */

typedef struct wsx_env wsx_env;   /* opaque host handle */

/* Policy model (App. B: deep policy models held in device memory, referenced
 * by every replica, never copied). Two tanh hidden layers and a linear head of
 * n_head = n_out + 1 rows whose last row is the value V(s).
 * Weights are [out][in] row-major in `dtype`: float for WSX_F32, bfloat16 bit
 * patterns for WSX_BF16, E4M3FN codes for WSX_FP8_E4M3 with real weight
 * s[out] * code. Biases are float. Products accumulate in FP32. */
typedef struct {
    int32_t dtype;           /* WSX_F32, WSX_BF16 or WSX_FP8_E4M3                 */
    int32_t d_in, h1, h2;    /* d_in = obs dim of the env kind; h1 == h2          */
    int32_t n_head;          /* outputs + 1 (value)                               */
    const void* w1;          /* device [h1][d_in]                                 */
    const void* w2;          /* device [h2][h1]                                   */
    const void* w3;          /* device [n_head][h2]                               */
    const float* b1;         /* device [h1]                                       */
    const float* b2;         /* device [h2]                                       */
    const float* b3;         /* device [n_head]                                   */
    const float* s1;         /* FP8: device [h1] power-of-two row scales, else NULL */
    const float* s2;         /* FP8: device [h2]                                  */
    const float* s3;         /* FP8: device [n_head]                              */
    float act_scale[3];      /* FP8: power-of-two scale of the obs, h1, h2 inputs */
    const float* log_std;    /* continuous kinds: device [n_head - 1], else NULL  */
} wsx_policy;

/* Trajectory buffers (App. B: roll-out data stored in place for training).
 * Slots [0, horizon) are written by wsx_rollout. Layout [T][rows] with
 * consecutive rows adjacent (obs: [T][rows][obs_dim]). */
typedef struct {
    int32_t capacity;        /* number of T slots allocated                       */
    float* obs;              /* observation before the step                       */
    void* action;            /* uint8 [T][rows] (discrete) or float (continuous)  */
    float* reward;
    uint8_t* done;           /* 1 if the transition terminated (auto-reset next)  */
    float* value;            /* V(s_t)                                            */
    float* logp;             /* log-probability of the action taken               */
    float* last_value;       /* [rows] V(s_T) of the state after the last step    */
} wsx_traj;

/* Size in bytes of the device state block an environment set needs (Sec. 2
 * and App. B: every replica's state lives in device memory for the whole
 * run): the state, per-step scratch for the PLAIN mode, for the market the
 * CSR offsets, the tile table and its row and slot maps, for the reaction
 * walk its FP64 energy terms. n_rows: agents (market) or n_envs. Errors:
 * WSX_EINVAL (unknown kind, n_envs <= 0, n_rows < n_envs, single-agent kinds
 * with n_rows != n_envs, NULL bytes), WSX_EUNSUPPORTED (n_rows >= 2^31). */
int wsx_env_state_bytes(int32_t kind, int64_t n_envs, int64_t n_rows, size_t* bytes);

typedef struct {
    int32_t kind;            /* WSX_CARTPOLE ... WSX_REACTION                     */
    int32_t tile_rows;       /* rows per workgroup tile (market: agents), 0 = the */
                             /* default; runs on the compiled kernel with the     */
                             /* fewest row slots >= tile_rows                     */
    int32_t waves;           /* wavefronts per workgroup, 0 = any / the default   */
    int32_t occupancy;       /* min wavefronts per SIMD of the fused kernel, 0 =  */
                             /* any / the default; (tile_rows, waves, occupancy)  */
                             /* must match a compiled kernel (else EUNSUPPORTED)  */
    int64_t n_envs;
    uint64_t seed;           /* Philox key                                        */
    void* state;             /* device, wsx_env_state_bytes bytes, caller-owned,  */
                             /* must stay valid until wsx_env_destroy             */
    const int32_t* agent_offsets; /* market: HOST [n_envs + 1] CSR offsets of the */
                             /* agents (copied into `state` at create), else NULL */
    const float* params;     /* reaction: DEVICE potential block (A[20][20],      */
                             /* centres[64][20], widths[64], amplitudes[64]),     */
                             /* referenced, not copied; else NULL                 */
} wsx_env_desc;

/* Creates the host handle of an environment set (App. B: each replica runs
 * independently; the market's agents interact within their environment).
 * For the market, uploads the offsets and the tile table synchronously on the
 * null stream (the only host-to-device copy the library makes). The state is
 * undefined until wsx_env_reset. */
int wsx_env_create(const wsx_env_desc* desc, wsx_env** out);

/* Resets every row (App. B: reset runs on the device): draws the initial
 * state from the Philox RESET stream at step 0 of `epoch` and sets the step
 * counter to 0. */
int wsx_env_reset(wsx_env* env, uint32_t epoch, void* stream);

/* Rolls every replica forward `horizon` steps (App. B; Sec. 2: no CPU-GPU
 * transfer): per step observe, policy forward, sample, store the record,
 * step the dynamics, auto-reset terminated rows; then V(s_T). The step
 * counter advances by `horizon`, so consecutive calls continue the same
 * random streams (rollout(a) then rollout(b) equals rollout(a + b)).
 * traj->capacity must be >= horizon. */
int wsx_rollout(wsx_env* env, const wsx_policy* policy, int32_t horizon,
                const wsx_traj* traj, int32_t mode, void* stream);

/* Number of rows, current step counter and epoch of an environment set
 * (App. B: the step counter and the reset epoch key each replica's random
 * streams). Any pointer may be NULL. Errors: WSX_EINVAL (env NULL). */
int wsx_env_info(const wsx_env* env, int64_t* n_rows, uint32_t* step, uint32_t* epoch);

/* Several environment sets in ONE persistent fused launch (App. B: many
 * environment instances advanced together, each in its own GPU blocks):
 * set i runs `horizon` steps with policies[i] into trajs[i], with the same
 * results as wsx_rollout(WSX_MODE_FUSED) of that set on a kernel with the
 * same waves (rows never interact across sets). 1 <= n <= 4 distinct sets
 * on one device; their kinds are one kind, or Pendulum and Acrobot together
 * (compiled pair kernels); the policies share dtype and width. The launch
 * uses the waves and occupancy of envs[0] and the smallest kernel that holds
 * every set's tile height. Each set's step counter advances by `horizon`.
 * Errors: WSX_EINVAL (arguments), WSX_EUNSUPPORTED (no kernel for the mix),
 * WSX_EHIP. */
int wsx_rollout_batch(wsx_env* const* envs, const wsx_policy* const* policies,
                      const wsx_traj* const* trajs, int32_t n, int32_t horizon, void* stream);

/* What a fused batch launch does besides the roll-out (wsx_rollout_batch_ext):
 * a reset before the first step and the returns/GAE after the last, in the
 * same kernel, so one launch runs a whole iteration of the hot path (Sec. 2:
 * simulation and data preparation for training stay on the device; Sec. 3:
 * actor-critic consumes returns and advantages). */
typedef struct {
    int32_t reset;           /* 1: every row first takes its initial state, as   */
                             /* wsx_env_reset(env, epoch) would draw it, and the */
                             /* step counter restarts at 0                       */
    uint32_t epoch;
    int32_t returns;         /* 1: returns and GAE of each set over the horizon,  */
                             /* the recursions of wsx_compute_returns (FP64)     */
    int32_t bootstrap;       /* as in wsx_compute_returns                         */
    int32_t out_dtype;       /* WSX_F32 or WSX_F64                                */
    double gamma, lambda;    /* in [0, 1]                                         */
    void* const* ret;        /* [n] device buffers [horizon][rows] of out_dtype   */
    void* const* adv;        /* [n] device buffers [horizon][rows]                */
} wsx_rollout_ext;

/* wsx_rollout_batch with a reset before and returns/GAE after the roll-out,
 * all in the one persistent launch: each workgroup resets its tile's rows
 * from the RESET stream (when ext->reset), rolls them out, and then computes
 * their returns and advantages from the records it has just written (FP64,
 * segments of the horizon composed as affine maps; equal to
 * wsx_compute_returns within FP64 rounding of the association order). The
 * trajectories and final states equal those of wsx_env_reset +
 * wsx_rollout_batch bit for bit. ext == NULL is wsx_rollout_batch. Buffers
 * are caller-owned; ret/adv must not overlap the trajectories. Errors:
 * WSX_EINVAL (as wsx_rollout_batch; NULL ret/adv when returns is set,
 * gamma/lambda outside [0, 1]), WSX_EUNSUPPORTED (out_dtype), WSX_EHIP. */
int wsx_rollout_batch_ext(wsx_env* const* envs, const wsx_policy* const* policies,
                          const wsx_traj* const* trajs, int32_t n, int32_t horizon,
                          const wsx_rollout_ext* ext, void* stream);

/* Workgroup tiles of an environment set's fused launch and the rows one tile
 * holds. Single-agent kinds: ceil(n_rows / tile_rows) tiles of consecutive
 * replicas. The market (App. B: the agents of one environment interact, so
 * they share one block): whole environments packed by first-fit decreasing
 * into tiles of at most `capacity` agents, so n_rows / (n_tiles * capacity)
 * is the tiles' fill. */
int wsx_env_tiles(const wsx_env* env, int32_t* n_tiles, int32_t* capacity);

/* Sets the step counter (resuming from a saved state block: App. B, the
 * roll-out continues in place). Errors: WSX_EINVAL (env NULL). */
int wsx_env_set_step(wsx_env* env, uint32_t step);

/* Steps per fused launch in WSX_MODE_FUSED_GRAPH (0 = the whole horizon in
 * one launch, the default); chunk_steps < 0 is WSX_EINVAL. Results do not
 * depend on it. */
int wsx_env_set_chunk(wsx_env* env, int32_t chunk_steps);

/* Releases the host handle and its cached graphs (App. B: the state stays in
 * device memory, owned by the caller, who frees the state block after this
 * call). Errors: WSX_EINVAL (env NULL). */
int wsx_env_destroy(wsx_env* env);

/* Discounted returns and GAE advantages (Sec. 3, actor-critic), FP64:
 *   delta_t = r_t + gamma (1 - d_t) V_{t+1} - V_t
 *   A_t = delta_t + gamma lambda (1 - d_t) A_{t+1}
 *   G_t = r_t + gamma (1 - d_t) G_{t+1}
 * with V_T = G_T = last_value[row] if bootstrap, else 0. Inputs are the
 * trajectory fields ([T][rows]); outputs [T][rows] in WSX_F32 or WSX_F64. */
int wsx_compute_returns(const float* reward, const float* value, const uint8_t* done,
                        const float* last_value, int32_t horizon, int64_t rows,
                        double gamma, double lambda, int32_t bootstrap,
                        void* returns, void* advantages, int32_t out_dtype, void* stream);

/* Policy forward alone (the inference step of App. B) for `rows`
 * observations [rows][d_in] float: head outputs [rows][n_head] float. Uses
 * the same device code and accumulation order as the roll-out kernels. */
int wsx_policy_forward(const wsx_policy* policy, const float* obs, int64_t rows,
                       float* head, void* stream);

/* Policy forward with the kernel of an environment set's roll-out (the same
 * weight split over waves and the same FP32 accumulation order as that set's
 * fused and plain launches, App. B's action inference), for `rows`
 * observations [rows][d_in] float: head outputs [rows][n_head] float, and the
 * quantised outputs of both hidden layers -- the inputs of the second and
 * third products -- as codes of the policy format, [rows][hidden] each:
 * bfloat16 (2 bytes), OCP E4M3 (1 byte; the value is code x act_scale[1] or
 * act_scale[2]) or float (FP32 policies). Lets a checker adopt the rounding
 * decisions the FP32 accumulation took next to a rounding midpoint and test
 * every other result tightly. act1 / act2 / head: caller-owned device
 * buffers. Built-in kinds only. Errors: WSX_EINVAL (NULL pointers, rows out
 * of range, policy shape not the set's), WSX_EUNSUPPORTED (user kinds),
 * WSX_EHIP. */
int wsx_policy_trace(const wsx_env* env, const wsx_policy* policy, const float* obs,
                     int64_t rows, float* head, void* act1, void* act2, void* stream);

/* Rounds n floats to `dtype` (WSX_BF16: RNE; WSX_FP8_E4M3: s * fp8(x / s),
 * RNE, saturating) with the device conversion the kernels use and returns
 * the real values as float: the quantisation points of the policy forward
 * (the paper runs policy inference on the device, App. B, and fixes no
 * precision; these formats are this library's). x, y: device [n] float,
 * caller-owned. Errors: WSX_EINVAL (unknown dtype, scale not a positive power
 * of two, n < 0, NULL pointers), WSX_EHIP. */
int wsx_quantize(int32_t dtype, float scale, const float* x, float* y, int64_t n, void* stream);

/* ------------------------------------------------------------------------ */
/* Actor-critic update on the roll-out data in place (Sec. 3: actor-critic  */
/* training for discrete and continuous actions; App. A: the trainer reads   */
/* the roll-out where it was written). The loss, averaged over `samples`     */
/* samples i (a trajectory's horizon x rows, its fields passed as flat       */
/* arrays), is                                                               */
/*   L = (1/n) sum_i [ -A_i log pi(a_i|o_i) + (value_coef/2) (V(o_i) - G_i)^2 */
/*                     - entropy_coef H(pi(.|o_i)) ]                         */
/* with A and G from wsx_compute_returns (WSX_F32 outputs). Gaussian         */
/* policies (log_std set): log pi = -(a - mu)^2 / (2 sigma^2) - log sigma -  */
/* log(2 pi)/2 with sigma = exp(log_std[0]); categorical: softmax of the     */
/* logits. The policy is evaluated as the roll-out evaluates it and the      */
/* rounding of its inputs is passed straight through (tanh' at the unrounded */
/* FP32 activation); for BF16 policies the operands of the backward products */
/* are rounded to BF16 (head gradient, dz2, dz1), bias gradients are not.    */
/* FP32 and BF16 policies of the compiled shapes (FP32 hidden 64, BF16 hidden */
/* 256; n_head <= 16, or <= 64 for BF16) -- else WSX_EUNSUPPORTED (FP8).     */
/* ------------------------------------------------------------------------ */

/* FP32 gradients, device, caller-owned, the policy's shapes and layouts. */
typedef struct {
    float* w1;               /* [h1][d_in]                                        */
    float* b1;               /* [h1]                                              */
    float* w2;               /* [h2][h1]                                          */
    float* b2;               /* [h2]                                              */
    float* w3;               /* [n_head][h2]                                      */
    float* b3;               /* [n_head]                                          */
    float* log_std;          /* [1] for Gaussian policies; ignored for categorical */
} wsx_grads;

/* Device workspace wsx_ac_grad needs for `samples` samples on the current
 * device: per sample of a chunk three rows of `h1` elements in the policy's
 * format, plus per-workgroup partial sums. Sets of more than 2^21 samples run
 * in chunks of 2^21, so the size stops growing there (about 3 GiB for a BF16
 * policy of width 256). */
int wsx_ac_grad_workspace_bytes(const wsx_policy* policy, int64_t samples, size_t* bytes);

/* Writes the gradient of L into `grads` (overwritten, not accumulated).
 * n_actions: K >= 2 for a categorical policy over K actions (n_head == K + 1,
 * action uint8), 0 for a Gaussian policy (n_head == 2, policy->log_std
 * required, action float). obs: device [samples][d_in] float; action
 * [samples]; returns, advantages: float [samples]. samples >= 1. The
 * workspace (device, at least wsx_ac_grad_workspace_bytes) is scratch for
 * the call; calls that share a workspace must be ordered on one stream. */
int wsx_ac_grad(const wsx_policy* policy, int32_t n_actions, const float* obs,
                const void* action, const float* returns, const float* advantages,
                int64_t samples, float value_coef, float entropy_coef,
                const wsx_grads* grads, void* workspace, size_t workspace_bytes, void* stream);

/* wsx_ac_grad without a workspace argument and without any allocation, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving or training loops, harnesses that forbid hipMalloc). The
 * workspace is a file-scope device array of the library (about 23 MiB, one
 * per GPU, held until the process ends), which bounds `samples` to
 * WSX_AC_STATIC_MAX_SAMPLES; larger counts return WSX_EINVAL, other errors
 * as wsx_ac_grad. Same arguments and results as wsx_ac_grad (the same kernels
 * and the same partial-sum layout, so the gradients are equal bit for bit).
 * Every call on a GPU shares that GPU's array: calls that overlap on one GPU
 * (other streams, other threads) race; order them on one stream. */
#define WSX_AC_STATIC_MAX_SAMPLES 2048
int wsx_ac_grad_static(const wsx_policy* policy, int32_t n_actions, const float* obs,
                       const void* action, const float* returns, const float* advantages,
                       int64_t samples, float value_coef, float entropy_coef,
                       const wsx_grads* grads, void* stream);

/* One Adam step (Kingma and Ba, ICLR 2015, Algorithm 1) on n FP32 master
 * parameters in place, step t >= 1 (bias corrections 1 - beta^t):
 *   m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
 *   p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
 * If `store` is not NULL the updated parameter is also written there in
 * store_dtype (WSX_F32, or WSX_BF16 rounded to nearest even): the policy's
 * own weight buffer, so the next roll-out uses the new weights. */
int wsx_adam_step(float* param, const float* grad, float* m, float* v, int64_t n, int32_t step,
                  float lr, float beta1, float beta2, float eps, void* store,
                  int32_t store_dtype, void* stream);

/* The same Adam step on several tensors in one launch (one step t and one set
 * of hyper-parameters): exactly wsx_adam_step on each tensor, for callers
 * that update a policy's weight tensors together. n_tensors in
 * 1..WSX_ADAM_MAX_TENSORS; each entry as wsx_adam_step's arguments (n >= 0;
 * entries with n == 0 are skipped; pointers of the others non-NULL). The
 * tensors must not overlap. */
#define WSX_ADAM_MAX_TENSORS 16
typedef struct {
    float* param;            /* n FP32 masters, updated in place                  */
    const float* grad;       /* n FP32 gradients                                  */
    float* m;                /* n FP32 first moments                              */
    float* v;                /* n FP32 second moments                             */
    int64_t n;
    void* store;             /* NULL, or n values in store_dtype                  */
    int32_t store_dtype;     /* WSX_F32 or WSX_BF16                               */
} wsx_adam_tensor;

int wsx_adam_step_many(const wsx_adam_tensor* tensors, int32_t n_tensors, int32_t step, float lr,
                       float beta1, float beta2, float eps, void* stream);

/* ------------------------------------------------------------------------ */
/* User environment kinds (Sec. 2: the framework is environment-agnostic;    */
/* App. B: user environments are compiled for the device and run in the same */
/* GPU-resident loop). `source` defines, in C++ for HIP, a `struct UserEnv`  */
/* with the interface of the built-in kinds:                                 */
/*   static constexpr int KIND = WSX_USER_KIND, SD, SR, OD, NACT, LANES;    */
/*     SD state floats per row kept in the state block, SR >= SD in          */
/*     registers, OD observation size, NACT actions (0: one continuous       */
/*     action), LANES lanes that may share a row (1 unless the step uses the */
/*     group reductions);                                                    */
/*   __device__ static void complete(float* s);   derived register entries   */
/*   __device__ static void reset(float* s, const RngKey& key, uint32_t t,   */
/*                                uint32_t row, const EnvCtx& ctx);          */
/*   __device__ static void observe(const float* s, float* o);               */
/*   template <int G> __device__ static void step(float* s, int a, float av, */
/*       uint32_t t, uint32_t row, const RngKey& key, const EnvCtx& ctx,     */
/*       int sub, float& reward, bool& done);                                */
/* It may use the library's device helpers (Philox `draw`, `unit_uniform`,   */
/* `sin_cos`, `wrap_pi`, ...). The call compiles the fused roll-out and the  */
/* reset kernel for it with the HIP run-time compiler for the current device */
/* (a second or so), loads them, and returns a new kind (>= 100) that works  */
/* with wsx_env_state_bytes, wsx_env_create (without agent_offsets and       */
/* params), wsx_env_reset, wsx_rollout in WSX_MODE_FUSED and                 */
/* WSX_MODE_FUSED_GRAPH, wsx_rollout_batch of sets of this kind, and the     */
/* returns and update calls. Policies: FP32 width 64 with <= 16 head         */
/* outputs, or BF16 width 256. A source that does not compile returns        */
/* WSX_EINVAL with the compiler's log in wsx_last_error(). The kernels are  */
/* loaded on the device current at registration; launching a kind while     */
/* another device is current returns WSX_EHIP. Kinds stay registered until  */
/* the process ends.                                                         */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t state_dim;       /* SD                                                */
    int32_t obs_dim;         /* OD                                                */
    int32_t n_actions;       /* NACT: 0, or 2..255                                */
    int32_t dtype;           /* policy format: WSX_F32 or WSX_BF16                */
    int32_t hidden;          /* policy width: 64 (FP32) or 256 (BF16)             */
} wsx_user_kind_desc;

int wsx_user_kind_register(const wsx_user_kind_desc* desc, const char* source, int32_t* kind);

/* ------------------------------------------------------------------------ */
/* Autotuner for the persistent fused roll-out (App. B: every environment    */
/* instance owns a GPU block, its agents the block's threads; here a tile of */
/* rows per workgroup, whose best height depends on the set). Times the      */
/* fused roll-out of one environment set on every compiled kernel shape      */
/* (rows per workgroup tile -- including tile heights that spread the rows   */
/* evenly over the compute units --, waves per workgroup, occupancy, hence   */
/* the weight registers per wave) and then the chunk length of the graph     */
/* mode, and records the fastest in the library's tuning table under (kind,  */
/* n_envs, n_rows, compute units). wsx_env_create with tile_rows, waves and  */
/* occupancy all 0 takes its shape and chunk from a matching table entry     */
/* (else the built-in default). The table is process-wide and thread-safe;   */
/* it persists only through wsx_tune_save / wsx_tune_load.                   */

typedef struct {
    int32_t tile_rows, waves, occupancy; /* the kernel shape                  */
    int32_t chunk_steps;     /* steps per launch in WSX_MODE_FUSED_GRAPH       */
    double us_per_step;      /* measured time of one step of the whole set     */
} wsx_tune_entry;

/* Bytes of device workspace wsx_autotune needs for this environment set (the
 * state block and a trajectory of `horizon` steps). desc->state is ignored. */
int wsx_autotune_workspace_bytes(const wsx_env_desc* desc, int32_t horizon, size_t* bytes);

/* Runs the search on `stream` and waits for it (it is a host-synchronous
 * call). desc->state is ignored; the workspace (device, caller-owned) holds
 * the trial state and trajectory. Each candidate runs one untimed roll-out of
 * `horizon` steps and `reps` (>= 1) timed ones; the median counts. `best`
 * (optional) receives the winner. Errors: WSX_EINVAL (arguments, workspace
 * too small, horizon < 1), WSX_EUNSUPPORTED (no kernel for the policy),
 * WSX_EHIP. */
int wsx_autotune(const wsx_env_desc* desc, const wsx_policy* policy, int32_t horizon,
                 int32_t reps, void* workspace, size_t workspace_bytes, wsx_tune_entry* best,
                 void* stream);

/* The same search for a batch of 1..4 environment sets run together by
 * wsx_rollout_batch (one shape for all: each set's tile height, waves and
 * occupancy); the winner is recorded for every set of the batch, so sets
 * created afterwards with the default shape run the batch on it. The
 * workspace holds every set's trial state and trajectory (the sum of
 * wsx_autotune_workspace_bytes, each rounded up to 256 bytes). */
int wsx_autotune_batch_workspace_bytes(const wsx_env_desc* const* descs, int32_t n,
                                       int32_t horizon, size_t* bytes);
int wsx_autotune_batch(const wsx_env_desc* const* descs, const wsx_policy* const* policies,
                       int32_t n, int32_t horizon, int32_t reps, void* workspace,
                       size_t workspace_bytes, wsx_tune_entry* best, void* stream);

/* The table entry for (kind, n_envs, n_rows, compute units): WSX_OK and *out
 * filled, or WSX_EINVAL if there is none. */
int wsx_tune_lookup(int32_t kind, int64_t n_envs, int64_t n_rows, int32_t cus,
                    wsx_tune_entry* out);

/* Writes the table as text (one entry per line: kind n_envs n_rows cus
 * tile_rows waves occupancy chunk_steps us_per_step) / merges such a file into
 * the table (later entries replace earlier ones with the same key). A line
 * that does not parse, or names no compiled kernel shape, is WSX_EINVAL and
 * nothing from the file is kept. */
int wsx_tune_save(const char* path);
int wsx_tune_load(const char* path);

/* The kernel shape and chunk length an environment set runs with (App. B: a
 * block per environment instance; here rows per workgroup tile, waves per
 * workgroup, occupancy). Any pointer may be NULL. Errors: WSX_EINVAL. */
int wsx_env_shape(const wsx_env* env, int32_t* tile_rows, int32_t* waves, int32_t* occupancy,
                  int32_t* chunk_steps);

/* ------------------------------------------------------------------------ */
/* Roll-out server: continuous batching of roll-out requests.                */
/* The paper has no serving layer: it keeps thousands of replicas and their  */
/* roll-out data resident on one GPU (Sec. 2, App. B). The server applies    */
/* that to a stream of independent requests.                                 */
/*                                                                          */
/* Requests (an environment kind, a number of replicas, a horizon, a policy) */
/* are submitted from any thread and run by a scheduler thread inside the    */
/* library. Memory for a request (its environment state block, trajectory    */
/* and returns) is sub-allocated from a caller-owned device arena, which is   */
/* the HBM admission budget: a request waits until its memory fits. The      */
/* scheduler advances every admitted request in rounds of at most            */
/* chunk_steps steps; each round issues, per (kind, policy), ONE fused       */
/* launch covering the tiles of all admitted requests of that kind, so a     */
/* request that arrives while others run joins the next round and shares    */
/* launches with them, and kinds run concurrently on separate streams. A     */
/* finished request gets its returns/GAE and its latency recorded.           */
/* Environment state is device-resident in sessions: a request may continue  */
/* a session left by an earlier request. Results do not depend on the mix:   */
/* a request's numbers equal those of the same roll-out run alone.           */
/* ------------------------------------------------------------------------ */

typedef struct wsx_server wsx_server;   /* opaque */

typedef struct {
    void* arena;             /* caller-owned device memory sub-allocated by the   */
    size_t arena_bytes;      /* server; its size is the admission budget          */
    int32_t chunk_steps;     /* steps per scheduling round (> 0)                   */
    int32_t max_batch;       /* most requests in one batched launch (> 0)          */
} wsx_server_desc;

typedef struct {
    int32_t kind;            /* WSX_PENDULUM ... (any kind)                        */
    int32_t horizon;         /* steps (> 0)                                        */
    int64_t n_envs;          /* replicas of a new session (ignored when continuing) */
    uint64_t seed;           /* Philox key of a new session                        */
    uint32_t epoch;          /* reset epoch of a new session                       */
    int32_t keep_session;    /* 1: keep the state resident after the request       */
    int64_t session;         /* 0: new session; else continue this session id      */
    const wsx_policy* policy;/* copied at submit; its device buffers must stay     */
                             /* valid until the request completes                  */
    const int32_t* agent_offsets; /* market, new session: HOST [n_envs + 1], copied */
    const float* params;     /* reaction, new session: DEVICE potential block      */
    double gamma, lambda;    /* returns / GAE parameters                           */
} wsx_request;

typedef struct {
    int32_t status;          /* 0 queued, 1 admitted, 2 done, < 0 failed (code)    */
    int32_t reserved;
    int64_t session;         /* the session the request ran in                     */
    int64_t n_rows;
    wsx_traj traj;           /* device pointers in the arena, valid until release  */
    float* returns;          /* device [horizon][rows] FP32 (FP64 arithmetic)      */
    float* advantages;
    double queue_ms;         /* submit -> admission                                */
    double latency_ms;       /* submit -> results complete on the device           */
} wsx_result;

typedef struct {
    int64_t submitted, admitted, completed, launches;
    int64_t env_steps;       /* completed replica-steps                            */
    size_t arena_in_use, arena_peak;
    int32_t queued, running;
} wsx_server_stats;

/* Creates the server and starts its scheduler thread (streams at default
 * priority are created on the current device). desc->arena: caller-owned
 * device memory, kept until wsx_server_destroy. Errors: WSX_EINVAL (NULL
 * arguments, empty arena, arena smaller than the launch tables,
 * chunk_steps or max_batch <= 0), WSX_EHIP. */
int wsx_server_create(const wsx_server_desc* desc, wsx_server** out);

/* Queues a request; returns its id. Fails with WSX_EINVAL if its memory can
 * never fit the arena or the arguments are invalid. */
int wsx_server_submit(wsx_server* srv, const wsx_request* req, int64_t* id);

/* Waits up to timeout_ms (< 0: forever) for request `id`; fills *out.
 * WSX_ETIMEOUT if it has not completed in time (then *out holds its state). */
int wsx_server_wait(wsx_server* srv, int64_t id, int32_t timeout_ms, wsx_result* out);

/* Frees a completed request's trajectory and returns (and its session unless
 * it was kept). Errors: WSX_EINVAL (unknown id), WSX_ESTATE (not completed). */
int wsx_server_release(wsx_server* srv, int64_t id);

/* Cancels a request: a queued one leaves the queue, a running one gets no
 * further rounds and ends once its rounds on the device have ended; either
 * way its status becomes WSX_ECANCELED (wsx_server_wait returns it) and its
 * memory is freed by wsx_server_release. Other requests are unaffected.
 * Errors: WSX_EINVAL (unknown id), WSX_ESTATE (already ended, or its last
 * round and returns are already on the device). */
int wsx_server_cancel(wsx_server* srv, int64_t id);

/* Test support for failure isolation (not an operation of the method):
 * marks request `id` so that its next launch is reported as failed. The
 * round's shared launch is then replaced by one launch per request, and
 * only the marked request ends, with WSX_EHIP, once its earlier rounds have
 * ended; the others run on. Errors: WSX_EINVAL (unknown id), WSX_ESTATE
 * (already ended). */
int wsx_server_inject_launch_failure(wsx_server* srv, int64_t id);

/* Frees a kept session that no request is using. Errors: WSX_EINVAL (unknown
 * session), WSX_ESTATE (a request is using it). */
int wsx_server_close_session(wsx_server* srv, int64_t session);

/* Counters of the server since its creation (requests, launches, replica
 * steps, arena use). Errors: WSX_EINVAL (NULL arguments). */
int wsx_server_get_stats(wsx_server* srv, wsx_server_stats* out);

/* Stops the scheduler after the device work in flight ends and frees the
 * server (the arena is the caller's). */
int wsx_server_destroy(wsx_server* srv);

/* Human-readable description of the last error on the calling thread
 * (thread-local, valid until the thread's next call into the library). */
const char* wsx_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* WSX_H */
