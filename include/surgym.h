/* surgym.h -- C interface of the MI355X batched serial-chain simulator.
 *
 * One context holds N independent environments, each a fixed-base serial
 * chain of revolute and prismatic joints driven by joint-space PD targets
 * (or C = 2 or 4 such chains sharing an episode), on one GPU. Beside the
 * step and the fused policy rollout it offers the learned dynamics
 * surrogate, step schedules for uneven joint counts, the PPO update of the
 * rollout policy and the adjoint of open-loop rollouts.
 * Every call enqueues work on the context's HIP stream and returns without
 * synchronizing; argument errors are reported synchronously.
 *
 * The method (paper: "Surgical Gym", Sec. III "Simulation Setup" and
 * "Policy learning and control"): physics, observations, rewards and the
 * policy rollout stay on the GPU and are exposed as device tensors, with a
 * Gym-like step (Sec. IV "Environments"). The dynamics are the textbook
 * ones of a contact-free serial chain (Featherstone 2008): RNEA bias
 * forces, the ABA articulated-inertia sweep, implicit PD drives folded in as
 * joint armature, semi-implicit Euler substeps, hard joint limits.
 *
 * Conventions shared by every call:
 *   N = n_env, J = max_dof (stride of per-joint arrays), W = 2*J + 10
 *   (observation width), T = rollout length.
 *   Device arrays are structure-of-arrays, env index fastest:
 *     per joint  [J][N]   element (j, e) at j*N + e
 *     obs        [W][N]   rows: q (J), qd (J), tip (3), goal (3),
 *                         goal - tip (3), |goal - tip| (1); unused joint
 *                         rows zero
 *   Element type "real" is float for SG_F32 contexts and double for SG_F64.
 *   Device pointers must be 16-byte aligned and hold the stated extents;
 *   the library never frees caller memory.
 *
 * Errors: every function returns sg_status. SG_E_INVAL: a null or
 * misaligned pointer, a size out of range; the message is available from
 * sg_last_error(ctx) (or sg_last_error(NULL) after a failed sg_create).
 * SG_E_UNSUPPORTED: a valid request the library does not implement (e.g. a
 * rollout on an FP64 context). SG_E_HIP: a HIP runtime error, including an
 * asynchronous fault surfaced at the next call that synchronizes.
 * A context is used by one host thread at a time.
 *
 * HIP graph capture: the device work of sg_step, sg_observe, sg_rollout,
 * sg_gae, the dynamics calls, sg_surrogate_train_step, sg_surrogate_predict,
 * sg_surrogate_step and sg_ppo_update is kernels only (no memset or memcpy
 * nodes), so a call can be captured on
 * the context's stream. The counters these calls advance live in device
 * memory and are advanced by the captured kernels themselves: the noise
 * counter (rng_step: the rollout's action noise, the tracking task's goal
 * draws) and the Adam step count of sg_ppo_update. Each replay of a
 * captured sg_step / sg_rollout / sg_surrogate_step therefore draws the next
 * steps' noise, each replay of a captured sg_ppo_update takes the next Adam
 * steps, exactly as the same number of eager calls would.
 */
#ifndef SURGYM_H
#define SURGYM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sg_ctx sg_ctx;

typedef enum {
  SG_OK = 0,
  SG_E_INVAL = -1,
  SG_E_UNSUPPORTED = -2,
  SG_E_HIP = -3,
  SG_E_STATE = -4,
  SG_E_NOMEM = -5
} sg_status;

enum { SG_F32 = 0, SG_F64 = 1 };
enum { SG_TASK_REACH = 0, SG_TASK_PATH = 1, SG_TASK_TRACK = 2 };
/* done flags (uint8 per env): bit 0 the episode ended (the observation
 * returned is the reset state's), bit 1 it ended by time-out (the critic
 * bootstraps, paper Sec. III "Policy learning and control"), bit 2 the
 * state went non-finite and was reset (reward 0). */
enum { SG_DONE_ENDED = 1, SG_DONE_TIMEOUT = 2, SG_DONE_NONFINITE = 4 };
/* armature for sg_forward_dynamics: none, or the implicit-PD drive's
 * h*kd + h^2*kp with h = dt / substeps. */
enum { SG_ARM_NONE = 0, SG_ARM_DRIVE = 1 };

enum { SG_JOINT_REVOLUTE = 0, SG_JOINT_PRISMATIC = 1 };

#define SG_MAX_DOF 16
#define SG_MAX_WAYPOINTS 32

/* Robot description. All arrays are HOST memory, float64, copied at
 * sg_create (values are rounded to the context's dtype there).
 * Chain geometry: joint j's origin is at offset_j in link j-1's frame (the
 * base frame for j = 0); link j's frame is that origin rotated by q_j about
 * the unit axis_j (revolute joint), or moved by q_j along axis_j without
 * rotation (prismatic joint; the paper's PSM and ECM arms each have one,
 * Sec. III "Robot Descriptions"). For a prismatic joint q is in m, kp in
 * N/m, kd in N s/m and limits in m. Joints j >= n_dof[e] of env e are
 * ignored; outputs hold 0 there. */
typedef struct {
  int32_t n_env;          /* N >= 1 */
  int32_t max_dof;        /* J, 1..SG_MAX_DOF */
  const int32_t* n_dof;   /* [N], 1..J */
  int32_t dtype;          /* SG_F32 or SG_F64 */
  const double* axis;     /* [3][J][N] unit joint axis */
  const double* offset;   /* [3][J][N] joint origin in the parent frame (m) */
  const double* com;      /* [3][J][N] link centre of mass, link frame (m) */
  const double* mass;     /* [J][N] > 0 (kg) */
  const double* inertia;  /* [6][J][N] xx yy zz xy xz yz about the COM, link axes */
  const double* kp;       /* [J][N] PD stiffness (N m / rad), >= 0 */
  const double* kd;       /* [J][N] PD damping (N m s / rad), >= 0 */
  const double* q_lo;     /* [J][N] lower joint limit (rad) */
  const double* q_hi;     /* [J][N] upper joint limit, > q_lo */
  const double* q0;       /* [J][N] reset position */
  const double* tip;      /* [3][N] tool tip in the last link's frame */
  double dt;              /* control period (s) > 0 */
  int32_t substeps;       /* S >= 1, substep h = dt / S */
  double gravity[3];      /* base-frame gravity (m/s^2) */
  const int32_t* joint_type; /* [J][N] SG_JOINT_REVOLUTE or SG_JOINT_PRISMATIC;
                              * NULL = all revolute. A context with any
                              * prismatic joint keeps the padded schedule and
                              * takes no surrogate (SG_E_UNSUPPORTED there). */
} sg_robot_desc;

/* Task description (paper Sec. IV): target reaching, reward -|tip - g|;
 * path following, reward -|tip - P(t)| with P(t) the waypoint
 * min(K-1, progress / dwell); or active tracking, reward -|tip - g_t| with a
 * moving goal: after each step that does not end the episode
 * g <- g + gd (held within +-offset of the episode centre per axis, the
 * outward velocity component dropped at the wall), then
 * gd <- gd + sigma N(0, 1); each new episode draws its centre as
 * track_centre + reset_std N(0, 1) per axis and starts the goal there at
 * rest (Philox counter (env, step, block 8 / 9) under `seed`). Rewards use
 * the goal active during the step; the observation holds the updated one.
 * Host memory, float64, copied at create. */
typedef struct {
  int32_t task;             /* SG_TASK_REACH, SG_TASK_PATH or SG_TASK_TRACK */
  int32_t n_waypoints;      /* K (path), 1..SG_MAX_WAYPOINTS */
  int32_t dwell;            /* control steps per waypoint (path), >= 1 */
  int32_t ep_len;           /* episode length in steps; <= 0: no time-out */
  const double* target;     /* [3][N] (reach; tracking: the first episode's centre) */
  const double* waypoints;  /* [K][3][N] (path) */
  const int32_t* progress0; /* [N] initial episode progress, may be NULL (0) */
  uint64_t seed;            /* noise key (exploration and the tracking goal) */
  double track_sigma;       /* tracking: goal-velocity increment std per step (m) */
  double track_offset;      /* tracking: half-width of the goal box (m), > 0 */
  double track_reset_std;   /* tracking: spread of a new episode's centre (m) */
  double track_centre[3];   /* tracking: nominal centre (m) */
  int32_t chains_per_env;   /* multi-tool reaching (Sec. IV): C = 1, 2 or 4
                             * consecutive env indices (chains) form one env;
                             * its reward is the sum of the chains' rewards
                             * (each toward its own goal), its episode is
                             * shared (progress0 equal within the group) and
                             * a non-finite chain resets all of them. Every
                             * output stays per chain (the reward repeated).
                             * 0 or 1: one chain per env. Tiled schedules
                             * need C = 1. */
  /* Per-episode re-randomisation (Sec. III: resets start new trajectories;
   * Sec. IV: targets and paths sampled per task instance), reach and path
   * tasks with one chain per env. At each reset the env draws its next
   * goal from Philox block 10 of (env, step) under `seed`: reach: target_k
   * = rand_centre_k + rand_half_width (2 u_k - 1) with u_k = ((word_k >> 8)
   * + 0.5) / 2^24, k = 0..2 (the first episode uses `target`); path: the
   * waypoint set floor((word_0 >> 8) n_banks / 2^24) of the n_banks sets in
   * `waypoints` [n_banks K][3][N] (the first episode uses set 0). The
   * current goal is the env's goal state (sg_get_goal_state). */
  int32_t rerandomize;      /* 0: goals fixed at create; 1: re-randomised */
  int32_t n_banks;          /* path: waypoint sets (1..64); 0 is taken as 1 */
  double rand_centre[3];    /* reach: centre of the target box (m) */
  double rand_half_width;   /* reach: half-width of the target box (m), > 0 */
} sg_task_desc;

/* Rollout storage, all DEVICE memory, float32 unless noted:
 *   obs [T+1][W][N]  obs[0] = observation before the first step
 *   act [T][J][N]    sampled (pre-clamp) actions
 *   logp, rew [T][N] log-density of act under the policy, reward
 *   done [T][N]      uint8 flags as above
 *   val [T+1][N]     critic value of obs[t]
 *   adv, ret [T][N]  GAE advantage and return */
typedef struct {
  float* obs;
  float* act;
  float* logp;
  float* rew;
  uint8_t* done;
  float* val;
  float* adv;
  float* ret;
  float gamma; /* discount, paper Sec. III (GAE) */
  float lam;   /* GAE lambda */
} sg_rollout_bufs;

/* Library version string. */
const char* sg_version(void);

/* Message of the last error on ctx (NULL: the calling thread's last
 * sg_create error). Never NULL. */
const char* sg_last_error(const sg_ctx* ctx);

/* Create N environments on the current HIP device. Copies the
 * descriptions, uploads them, and sets the state to (q0, 0, progress0),
 * noise step counter 0. *out receives the context. */
sg_status sg_create(const sg_robot_desc* robot, const sg_task_desc* task, sg_ctx** out);

/* Free the context and its device memory (after draining its stream). */
void sg_destroy(sg_ctx* ctx);

/* Bind the HIP stream (hipStream_t passed as void*; NULL = default). */
sg_status sg_set_stream(sg_ctx* ctx, void* hip_stream);

/* Wait for the context's stream; reports asynchronous HIP errors. */
sg_status sg_synchronize(sg_ctx* ctx);

/* Reset every env to (q0, 0, progress0), the tracking goals to their values
 * at create, and the noise counter to 0. */
sg_status sg_reset(sg_ctx* ctx);

/* One control step of every env (paper Sec. III: actions are PD position
 * targets, the solver advances in substeps; Sec. IV rewards):
 *   q* = mid + half_range * clamp(a, -1, 1) over the joint limits, held over
 *   S substeps of tau = kp (q* - q - h qd) - kd qd with armature
 *   h kd + h^2 kp, forward dynamics, qd += h qdd, q += h qd, hard limits;
 *   then tip position, reward, progress, time-out / non-finite reset, and
 *   the observation of the post-reset state.
 * actions [J][N] real (device), obs [W][N] real, reward [N] real,
 * done [N] uint8 (device). obs, reward, done may not alias actions. */
sg_status sg_step(sg_ctx* ctx, const void* actions, void* obs, void* reward, uint8_t* done);
/* (sg_step and sg_surrogate_step advance the noise counter rng_step by one,
 * sg_rollout by T; the counter is device memory, see HIP graph capture.) */

/* Step schedules for batches of uneven DOF (envs differ in n_dof). The
 * results do not depend on the schedule.
 *   SG_SCHED_PADDED     one launch, env order, every env padded to max_dof
 *                       with per-joint guards (the default);
 *   SG_SCHED_SORTED     one launch over 64-env tiles of one DOF class each
 *                       (tiles built at create), class-specialised code;
 *   SG_SCHED_PER_CLASS  the same tiles, one launch per DOF class;
 *   SG_SCHED_PERSISTENT the same tiles walked by at most 512 resident
 *                       blocks in one launch.
 * Tiled schedules are available on FP32 contexts without prismatic joints. */
enum { SG_SCHED_PADDED = 0, SG_SCHED_SORTED = 1, SG_SCHED_PER_CLASS = 2, SG_SCHED_PERSISTENT = 3 };
sg_status sg_set_schedule(sg_ctx* ctx, int32_t schedule);
sg_status sg_get_schedule(const sg_ctx* ctx, int32_t* schedule);

/* Mapping of the forward-dynamics solve onto waves (ABA, Featherstone
 * Table 7.1; the step of Sec. III): waves = 1, one env per lane and one wave
 * per 64 envs runs the whole solve; waves = 4, a wave team: the 64 envs'
 * workgroup has four waves, wave 0 keeps the state and runs the serial
 * recursions, and link j's inertia rotation and bias force (pass 1) run in
 * wave j mod 4, exchanged through LDS (the four waves also stage the
 * block's parameters together). The same operations in other waves: the
 * results agree with the one-wave solve to FP32 rounding. waves = 0 (the
 * default): the library picks: the team in sg_rollout, and in sg_step while
 * the launch's blocks all fit at once (N <= 128 x compute units: a team
 * block takes 62 KB of LDS, two per compute unit), one wave beyond. The
 * team runs in sg_step's padded schedule for chains of 4 to 9 joints and in
 * sg_rollout for chains of 4 to 7 joints with the 256-128 policy (the
 * Table II network's weight image leaves no LDS for the exchange);
 * elsewhere, and on FP64 contexts, the one-wave kernels run. SG_E_INVAL for
 * other values, SG_E_UNSUPPORTED for 4 on an FP64 context. */
sg_status sg_set_team(sg_ctx* ctx, int32_t waves);
sg_status sg_get_team(const sg_ctx* ctx, int32_t* waves);

/* Autotuner: time `trials` steps (after one warm-up) of every available
 * candidate with the given actions [J][N] (device), restoring the state
 * after each, and make the fastest the context's schedule and mapping.
 * Candidates, in the order of ms_per_step (host float[5], -1 for
 * unavailable; may be NULL): padded, sorted, per-class, persistent (one wave
 * per 64 envs), and padded with a wave team (sg_set_team; FP32 chains of 4
 * to 9 joints). *best gets the schedule, *best_team the waves per block
 * (either may be NULL). The choice is remembered for the rest of the
 * process under the context's key (device architecture, N, number type,
 * max joints, prismatic joints, chains per env, task, histogram of joint
 * counts): sg_create of a context with the same key starts from it.
 * Synchronizes the context's stream. */
sg_status sg_autotune_step(sg_ctx* ctx, const void* actions, int32_t trials, int32_t* best, int32_t* best_team,
                           float* ms_per_step);

/* The remembered autotuner choices as text, one line per key: the key, the
 * schedule and the waves per block, separated by spaces; for a caller to
 * store and hand to sg_tuning_import in a later process. Writes at most cap
 * bytes including the terminating 0 into buf (cap 0: none; buf may then be
 * NULL) and sets *len to the full length including the 0. sg_tuning_import
 * merges such lines into the process's choices (later lines win); a
 * malformed line gives SG_E_INVAL, the lines before it stay merged. */
sg_status sg_tuning_export(char* buf, size_t cap, size_t* len);
sg_status sg_tuning_import(const char* text);

/* Observation of the current state, obs [W][N] real (device). */
sg_status sg_observe(sg_ctx* ctx, void* obs);

/* Copy state out / in. q, qd [J][N] real and progress [N] int32 are device
 * pointers (any may be NULL to skip); rng_step is host memory
 * (sg_get_state with rng_step non-NULL copies the device counter out and
 * synchronizes the stream; sg_set_state enqueues a kernel that sets it). */
sg_status sg_get_state(sg_ctx* ctx, void* q, void* qd, int32_t* progress, uint64_t* rng_step);
sg_status sg_set_state(sg_ctx* ctx, const void* q, const void* qd, const int32_t* progress, uint64_t rng_step);
/* An env's mutable goal state (device, context dtype): tracking [9][N] =
 * goal (3), goal velocity (3), episode centre (3); re-randomised reach
 * [3][N] = the episode's target; re-randomised path [1][N] = the index of
 * the episode's waypoint set (an integer held as a real). SG_E_STATE for
 * tasks without one. */
sg_status sg_get_goal_state(sg_ctx* ctx, void* goal_state);
sg_status sg_set_goal_state(sg_ctx* ctx, const void* goal_state);

/* Forward dynamics (ABA, Featherstone Table 7.1) for the given state:
 * qdd = (H(q) + diag(arm))^-1 (tau - C(q, qd)) with arm per arm_mode.
 * q, qd, tau, qdd [J][N] real (device). */
sg_status sg_forward_dynamics(sg_ctx* ctx, const void* q, const void* qd, const void* tau, int32_t arm_mode,
                              void* qdd);

/* Inverse dynamics (RNEA, Featherstone Table 5.1): tau = H qdd + C.
 * q, qd, qdd, tau [J][N] real (device). */
sg_status sg_inverse_dynamics(sg_ctx* ctx, const void* q, const void* qd, const void* qdd, void* tau);

/* Tool-tip position (forward kinematics) tip [3][N] real for q [J][N]. */
sg_status sg_tip_position(sg_ctx* ctx, const void* q, void* tip);

/* Architecture of the rollout policy: W -> hidden[0] -> .. ->
 * hidden[n_hidden-1] -> J+1, hidden units tanh or ELU (z for z > 0, e^z - 1
 * otherwise); outputs 0..J-1 are the action mean, output J the critic
 * value. The library builds two networks: n_hidden = 2, hidden = {256, 128},
 * tanh (the path-following rollout's policy), and n_hidden = 3, hidden =
 * {256, 128, 64}, ELU (the network of the paper's Sec. IV Table II
 * learning-dynamics benchmark; all-revolute chains). */
typedef enum { SG_ACT_TANH = 0, SG_ACT_ELU = 1 } sg_activation;
typedef struct {
  int32_t n_hidden;   /* 2 or 3 */
  int32_t hidden[3];  /* layer widths */
  int32_t act;        /* sg_activation */
} sg_policy_arch;

/* Policy of the rollout (architecture arch, HOST). w_bf16: HOST, BF16 bit
 * patterns of every layer's W [out][in] concatenated row-major (W1 [h1][W],
 * W2 [h2][h1], (W3 [h3][h2],) Wo [J+1][h_last]); bias: HOST float32, every
 * layer's b concatenated the same way; log_std: HOST float32 [J]. J <= 7,
 * FP32 contexts; an architecture the library does not build returns
 * SG_E_UNSUPPORTED. Synchronizes. */
sg_status sg_set_policy(sg_ctx* ctx, const sg_policy_arch* arch, const uint16_t* w_bf16, const float* bias,
                        const float* log_std);

/* The policy network alone on n inputs: x [W][n] float32 (device),
 * out [J+1][n] float32 (device). BF16 matrix-core products with FP32
 * accumulation; each layer's input is rounded to BF16 (nearest, ties even). */
sg_status sg_policy_forward(sg_ctx* ctx, const float* x, int32_t n, float* out);

/* T-step rollout (paper Sec. III "Policy learning and control"): for each
 * step the policy gives mean mu and value V of the current observation;
 * the action a = mu + exp(log_std) * eps with eps standard normal from
 * Philox4x32-10 keyed by the seed, counter (env, step lo, step hi, joint
 * block) and Box-Muller; the env steps on clamp(a); after T steps V of the
 * last observation, then GAE with the time-out bootstrap
 * r += gamma * V(s_t) on time-outs. The noise step counter advances by T.
 * FP32 contexts with a policy set. 1 <= T <= 4096. */
sg_status sg_rollout(sg_ctx* ctx, int32_t T, const sg_rollout_bufs* bufs);

/* GAE backward scan alone (Schulman et al., cited in paper Sec. III) on
 * device float32 rew [T][N], val [T+1][N], uint8 done [T][N] ->
 * adv, ret [T][N]; n = number of envs (columns). */
sg_status sg_gae(sg_ctx* ctx, int32_t T, int32_t n, const float* rew, const float* val, const uint8_t* done,
                 float gamma, float lam, float* adv, float* ret);

/* ---- learned forward-dynamics surrogate -------------------------------
 * An ELU MLP 13J -> 256 -> 256 -> 256 -> J (J <= 7, FP32 contexts) predicts
 * the implicit-PD substep's joint accelerations from q, qd, tau~ and the 10
 * standard inertial parameters of every link (m, m c, rotational inertia
 * about the link origin xx yy zz xy xz yz), with z-scored inputs and
 * outputs. Matrix products use BF16 operands and FP32 accumulation on the
 * matrix cores; training keeps FP32 master weights (Adam). A prediction is
 * accepted when |RNEA(q, qd, qdd_hat) + arm qdd_hat - tau~| /
 * max(|tau~|, 1e-3) <= threshold, else the env is solved exactly (ABA).
 * Training samples are device arrays q, qd, tau, qdd [J][n_total] float32 and
 * env [n_total] int32 (the context env whose link parameters apply); a batch
 * selects rows idx [batch] (NULL: the first batch rows). A sample id out of
 * range gives an all-zero feature row and no loss or gradient contribution
 * (it still counts in the batch size); an env id out of range gives an
 * all-zero feature row. Neither is used to read memory. */
typedef struct sg_surrogate sg_surrogate;

/* Create a surrogate bound to ctx (its link parameters, stream and state);
 * max_batch bounds training batches (1..4M). */
sg_status sg_surrogate_create(sg_ctx* ctx, int32_t max_batch, sg_surrogate** out);
void sg_surrogate_destroy(sg_surrogate* s);

/* HOST float32 parameters packed per layer as W [out][in] row-major then
 * b [out] (sizes 13J, 256, 256, 256, J); norm: HOST float32
 * mu_x[13J] sd_x[13J] mu_y[J] sd_y[J], or NULL to keep the current one.
 * Resets the Adam state. */
sg_status sg_surrogate_set_params(sg_surrogate* s, const float* params, const float* norm);
sg_status sg_surrogate_get_params(sg_surrogate* s, float* params, float* norm);

/* Fit the normalisation (mean, std per input feature and output) to n
 * samples (device arrays as above). */
sg_status sg_surrogate_fit_norm(sg_surrogate* s, const float* q, const float* qd, const float* tau, const int32_t* env,
                                const float* qdd, int32_t n);

/* Mean squared error on normalised targets over a batch and its gradient
 * (device float32, packed like the parameters); loss: device float. */
sg_status sg_surrogate_grad(sg_surrogate* s, const float* q, const float* qd, const float* tau, const int32_t* env,
                            const float* qdd, int32_t n_total, const int32_t* idx, int32_t batch, float* grad,
                            float* loss);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on a
 * batch; loss (device float, may be NULL) receives the batch loss. */
sg_status sg_surrogate_train_step(sg_surrogate* s, const float* q, const float* qd, const float* tau,
                                  const int32_t* env, const float* qdd, int32_t n_total, const int32_t* idx,
                                  int32_t batch, float lr, float* loss);

/* Predicted accelerations qdd_hat [J][n] (device) for n samples. */
sg_status sg_surrogate_predict(sg_surrogate* s, const float* q, const float* qd, const float* tau, const int32_t* env,
                               int32_t n, float* qdd_hat);

/* One control step of the bound context (same contract as sg_step) with the
 * surrogate in every substep and the exact solve for the envs whose
 * residual exceeds threshold; n_fallback: device int32 [substeps] (may be
 * NULL) receives the number of exact solves per substep. */
sg_status sg_surrogate_step(sg_surrogate* s, const float* actions, float* obs, float* reward, uint8_t* done,
                            float threshold, int32_t* n_fallback);

/* ---- Differentiation ----------------------------------------------------
 * Adjoint of an open-loop rollout of T control steps from the context's
 * current state (left unchanged) with actions [T][J][N] (DEVICE float32):
 * loss [N] = sum_t |tip(q_{t+1}) - goal_t| (the negated reward sum of
 * paper Sec. IV's reaching / path-following tasks), g_act [T][J][N] = dL/da
 * (0 for saturated actions |a| >= 1) and g_mass [J][N] = dL/dm for each
 * link's mass with its geometry fixed (all of its inertial parameters scale
 * with m). The state is checkpointed every K steps (1 <= K <= T) and each
 * segment is recomputed (its substep states and accelerations kept for the
 * reverse sweep); a clamped coordinate passes no
 * gradient, and an episode that ends inside the rollout cuts the gradient
 * at its reset. FP32 contexts with max_dof <= 7. The library keeps a
 * workspace of sg_adjoint_workspace_bytes(T, K) per context, (re)allocated
 * on first use of a larger size (that call synchronizes the stream). */
sg_status sg_adjoint(sg_ctx* ctx, int32_t T, int32_t K, const float* actions, float* loss, float* g_act,
                     float* g_mass);
/* sg_adjoint for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving or training loops, harnesses that forbid
 * hipMalloc): the same computation, arguments, errors and results, with the
 * checkpoints and segment tape in a fixed library workspace of 16 MiB
 * (16,777,216 bytes) per GPU, a static device array held until the process
 * ends. No call allocates or frees memory. A (T, K) whose
 * sg_adjoint_workspace_bytes exceeds 16 MiB returns SG_E_INVAL before any
 * work is enqueued (at 4096 envs x 7 DOF x 4 substeps, T = 64 with K = 8
 * needs 14.0 MB). Every call on one GPU shares that GPU's workspace: calls
 * that overlap in time on one GPU (two streams, two host threads) race and
 * must be serialized by the caller; calls in one stream order are safe. The
 * workspace needs no clearing (every entry is written before it is read). */
sg_status sg_adjoint_static(sg_ctx* ctx, int32_t T, int32_t K, const float* actions, float* loss, float* g_act,
                            float* g_mass);
/* Device workspace sg_adjoint needs for (T, K), in bytes; -1 if invalid. */
int64_t sg_adjoint_workspace_bytes(const sg_ctx* ctx, int32_t T, int32_t K);
/* Replace the link masses by masses [J][N] (DEVICE, context dtype), scaling
 * each link's first moment and rotational inertia with it (geometry fixed). */
sg_status sg_set_link_masses(sg_ctx* ctx, const void* masses);

/* ---- PPO update (paper Sec. III "Policy learning and control": the GPU
 * PPO of Rudin et al.; clipped surrogate objective of Schulman et al.) ----
 * Trains the rollout policy of the bound context from its rollout buffers:
 * advantages normalised over the batch (mean, unbiased std + 1e-8); per
 * minibatch L = L_pi + value_coef L_v - entropy_coef H with
 *   L_pi = -mean(min(r A, clip(r, 1 - clip, 1 + clip) A)), r = pi / pi_old,
 *   L_v  = mean(max((V - R)^2, (V_old + clip(V - V_old, +-clip) - R)^2)),
 *   H    = sum_j (log_std_j + 0.5 + 0.5 log 2 pi);
 * gradient through the network (BF16 matrix products, FP32 accumulation,
 * FP32 master weights), global-norm clip, Adam. Every call is asynchronous
 * on the context's stream; results are deterministic for given inputs. */
typedef struct sg_ppo sg_ppo;

typedef struct {
  float clip;           /* ratio and value clip, > 0 (0.2) */
  float value_coef;     /* >= 0 (1.0) */
  float entropy_coef;   /* (0.01) */
  float max_grad_norm;  /* global gradient-norm bound; <= 0: none (1.0) */
  float lr, beta1, beta2, adam_eps;  /* Adam (1e-3, 0.9, 0.999, 1e-8) */
  int32_t epochs;       /* passes over the batch, >= 1 (5) */
  int32_t minibatches;  /* per pass, >= 1, dividing T N (4) */
} sg_ppo_config;

/* Create a trainer bound to an FP32 context (J <= 7) for a policy of
 * architecture arch (as in sg_set_policy) with initial FP32 parameters
 * params (HOST, flat: per layer W [out][in] then b [out] -- W1, b1, W2, b2,
 * (W3, b3,) Wo, bo -- then log_std [J]; W = 2 J + 10). The context's
 * rollout policy is set to them (BF16, round to nearest even). max_samples
 * bounds T N of later calls (1..16M). Synchronizes. */
sg_status sg_ppo_create(sg_ctx* ctx, const sg_policy_arch* arch, const float* params, int32_t max_samples,
                        sg_ppo** out);
void sg_ppo_destroy(sg_ppo* ppo);
/* Number of parameters P of the flat vector. */
int32_t sg_ppo_param_count(const sg_ppo* ppo);
/* Current master parameters into params (HOST float[P]); synchronizes. */
sg_status sg_ppo_get_params(sg_ppo* ppo, float* params);

/* Gradient of L over one minibatch of `rows` samples of a T-step rollout
 * (sample s = t N + env; idx: DEVICE int32 [rows] sample ids, or NULL for
 * 0..rows-1; an id outside [0, T N) gives a zero input row and no loss or
 * gradient contribution, though it counts in the minibatch size), with
 * advantages normalised over all T N samples first, the
 * entropy term included and no norm clip: grad DEVICE float[P]. stats
 * (DEVICE float[8], may be NULL): loss_pi, loss_v, entropy, approx_kl
 * (mean log pi_old - log pi), clip fraction, |grad|. */
sg_status sg_ppo_grad(sg_ppo* ppo, const sg_rollout_bufs* bufs, int32_t T, const int32_t* idx, int32_t rows,
                      const sg_ppo_config* cfg, float* grad, float* stats);

/* One PPO update on a T-step rollout: cfg->epochs passes; pass ep visits
 * the samples perm[ep T N .. (ep + 1) T N) (DEVICE int32, a permutation of
 * 0..T N - 1 per pass; NULL: in order) cut into cfg->minibatches
 * minibatches; each takes a clipped Adam step. Then the context's rollout
 * policy is rewritten from the updated parameters. stats (DEVICE float[8],
 * may be NULL): the sg_ppo_grad statistics averaged over the minibatches. */
sg_status sg_ppo_update(sg_ppo* ppo, const sg_rollout_bufs* bufs, int32_t T, const sg_ppo_config* cfg,
                        const int32_t* perm, float* stats);

/* ---- Measured device peaks ----
 * Times microkernels on the current device and stream 0 and returns (HOST
 * doubles) the FP32 vector FMA rate without packed-FP32 instructions over
 * the whole chip (TFLOP/s, 16 independent FMA chains per lane, two waves
 * per SIMD) and for one wave alone on its SIMD (GFLOP/s per wave, the same
 * FMA stream), the BF16 16x16x32 matrix-core rate (TFLOP/s) and a 1 GiB
 * device-to-device copy rate (read + write bytes, GB/s). Allocates 2 GiB
 * for the duration of the call; synchronizes. For context beside the
 * datasheet peaks a roofline fraction is quoted against. */
sg_status sg_measure_peaks(double* fp32_fma_tflops, double* fp32_fma_wave_gflops, double* bf16_mfma_tflops,
                           double* copy_gbps);

#ifdef __cplusplus
}
#endif

#endif /* SURGYM_H */
