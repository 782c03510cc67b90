// Test infrastructure: part of the FP64 CPU oracle. Only tests/, the smoke
// check and the CPU-baseline leg of the benchmark may load or run anything
// under oracle/; the product path never does.
//
// One control step of one environment: PD action mapping, S substeps of
// implicit-PD forward dynamics with semi-implicit Euler and joint-limit
// projection, then forward kinematics into reward, episode bookkeeping,
// auto-reset and the observation vector.
//
// Paper passages this follows: actions are PD position targets (Sec. III
// "Action Space", and joints accept PD targets per Sec. III "Simulation
// Setup"); the solver advances in substeps (Sec. III "Simulation Setup");
// the observation concatenates joint positions, velocities, the tool-tip
// position and the goal (Sec. III "Observation Space"); the target-reaching
// reward rho * ||eta_t - g|| and the path-following reward
// -alpha * ||eta_t - P(t)|| (Sec. IV "Environments"); time-outs are told
// apart from terminations so the critic can bootstrap (Sec. III "Policy
// learning and control"). Readings where the paper is silent:
//   * PD drive, implicit: tau~ = kp (q* - q - h qd) - kd qd with armature
//     arm = h kd + h^2 kp added to the joint inertia, which is exactly
//     tau = kp (q* - q') - kd qd' on the end-of-substep state;
//   * q* = mid + half_range * clamp(a, -1, 1) over the joint limits, held
//     constant over the substeps;
//   * hard-stop limits after each position update: q clamped, the outward
//     velocity component zeroed (q == hi counts as inside);
//   * rho = alpha = -1 / 1 (reward = minus the distance), on the post-step
//     tip; path waypoint index k = min(K-1, progress_before / dwell);
//   * episode end at progress == ep_len (bits 0|1: ended, time-out), a
//     non-finite state ends the episode too (bits 0|2) with reward 0; both
//     auto-reset to (q0, 0), progress 0; the observation returned is the
//     post-reset one;
//   * observation (width 2*Jmax + 10): [q (Jmax), qd (Jmax), tip (3),
//     goal (3), goal - tip (3), |goal - tip| (1)], unused joint slots zero.
#pragma once
#include <cmath>
#include <cstdint>

#include "chain.hpp"
#include "rl.hpp"

namespace ora {

enum { kTaskReach = 0, kTaskPath = 1, kTaskTrack = 2 };
// Philox blocks of the tracking task's draws (the action noise uses blocks
// 0..3 of the same (env, step) counter).
enum { kBlockGoalAccel = 8, kBlockGoalReset = 9 };
// Philox block of the per-episode re-randomisation draw (reach, path).
enum { kBlockRerand = 10 };
enum { kDoneEnded = 1, kDoneTimeout = 2, kDoneNonFinite = 4 };

template <class T> struct Drive {
  T kp[kMaxDof], kd[kMaxDof], lo[kMaxDof], hi[kMaxDof], q0[kMaxDof];
};

struct TaskSpec {
  int task;         // kTaskReach, kTaskPath or kTaskTrack
  int n_waypoints;  // K (path task)
  int dwell;        // control steps per waypoint (path task)
  int ep_len;       // episode length in control steps; <= 0: never times out
  // active tracking (paper Sec. IV): goal random walk g += gd,
  // gd += sigma N(0, 1) per step; |g - centre| <= offset per axis; at each
  // reset a new centre = (cx, cy, cz) + reset_std N(0, 1) per axis
  double trk_sigma, trk_offset, trk_reset_std, trk_centre[3];
  // multi-tool reaching (paper Sec. IV): C consecutive chains form one env
  int chains = 1;
  // per-episode re-randomisation (reach and path, one chain per env): each
  // new episode draws its target in the box centre +- half per axis (reach)
  // or one of the n_banks waypoint sets (path; wp_all [n_banks K][3][N])
  int rerand = 0, n_banks = 1, N = 0;
  double rand_centre[3] = {0, 0, 0}, rand_half = 0;
  const double* wp_all = nullptr;
};

// Moving goal of one env (tracking task): position, velocity (per control
// step) and the episode's centre.
template <class T> struct Track {
  V3<T> g, gd, gc;
};

// Goal update of the tracking task after a step that did not end the
// episode: position by the velocity, clamp to the offset box (the outward
// velocity component is dropped at the wall), then the velocity's random
// increment.
template <class T>
inline void track_advance(const TaskSpec& ts, Track<T>& tr, uint64_t seed, uint32_t env, uint64_t step) {
  T* g = &tr.g.x;
  T* gd = &tr.gd.x;
  const T* gc = &tr.gc.x;
  double n4[4];
  gaussian_block(seed, env, step, kBlockGoalAccel, n4);
  for (int k = 0; k < 3; ++k) {
    g[k] = g[k] + gd[k];
    const T hi = gc[k] + T(ts.trk_offset), lo = gc[k] - T(ts.trk_offset);
    if (g[k] > hi) {
      g[k] = hi;
      if (gd[k] > T(0.0)) gd[k] = T(0.0);
    } else if (g[k] < lo) {
      g[k] = lo;
      if (gd[k] < T(0.0)) gd[k] = T(0.0);
    }
    gd[k] = gd[k] + T(ts.trk_sigma * n4[k]);
  }
}

// New episode of the tracking task: a new centre, the goal on it, at rest.
template <class T>
inline void track_reset(const TaskSpec& ts, Track<T>& tr, uint64_t seed, uint32_t env, uint64_t step) {
  double n4[4];
  gaussian_block(seed, env, step, kBlockGoalReset, n4);
  T* gc = &tr.gc.x;
  for (int k = 0; k < 3; ++k) gc[k] = T(ts.trk_centre[k] + ts.trk_reset_std * n4[k]);
  tr.g = tr.gc;
  tr.gd = v3(T(0.0), T(0.0), T(0.0));
}

template <class T> struct EnvGoal {
  V3<T> target;       // reach task
  V3<T> wp[32];       // path task waypoints
};

// Per-env episode goal under re-randomisation: the reach target, or the
// index of the path's waypoint set.
template <class T> struct Rerand {
  V3<T> target;
  int bank = 0;
};

// The goal of the episode rr describes, into g (env = its column).
template <class T> inline void apply_rerand(const TaskSpec& ts, const Rerand<T>& rr, int env, EnvGoal<T>& g) {
  if (ts.task == kTaskReach) {
    g.target = rr.target;
  } else {
    for (int k = 0; k < ts.n_waypoints; ++k) {
      const double* w = ts.wp_all + ((size_t)rr.bank * ts.n_waypoints + k) * 3 * ts.N;
      g.wp[k] = v3(T(w[0 * ts.N + env]), T(w[1 * ts.N + env]), T(w[2 * ts.N + env]));
    }
  }
}

// A new episode's goal (paper Sec. III: resets start new trajectories; Sec.
// IV: targets and paths are sampled per task instance): from the four words
// of Philox block kBlockRerand of (env, step): reach: 24-bit uniforms u_k,
// target_k = centre_k + half (2 u_k - 1), k = 0..2; path: the set
// floor(m n_banks / 2^24) with m = word 0 >> 8 (integer arithmetic, so
// every implementation picks the same set).
template <class T>
inline void rerand_reset(const TaskSpec& ts, Rerand<T>& rr, uint64_t seed, uint32_t env, uint64_t step) {
  Philox4 c = {{env, (uint32_t)step, (uint32_t)(step >> 32), (uint32_t)kBlockRerand}};
  const Philox4 x = philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  if (ts.task == kTaskReach) {
    T* t = &rr.target.x;
    for (int k = 0; k < 3; ++k) t[k] = T(ts.rand_centre[k] + ts.rand_half * (2.0 * u24(x.v[k]) - 1.0));
  } else {
    rr.bank = (int)(((uint64_t)(x.v[0] >> 8) * (uint64_t)ts.n_banks) >> 24);
  }
}

template <class T> inline V3<T> goal_for(const TaskSpec& ts, const EnvGoal<T>& g, int progress) {
  if (ts.task == kTaskReach) return g.target;
  int k = progress / ts.dwell;
  if (k > ts.n_waypoints - 1) k = ts.n_waypoints - 1;
  return g.wp[k];
}

// Physics part of a control step (substeps only). qdd_log, if non-null,
// receives the joint accelerations of every substep ([S][n]).
template <class T>
inline void physics_step(const Chain<T>& ch, const Drive<T>& dr, T dt, int S, const T* action, T* q, T* qd,
                         T* qdd_log) {
  const int n = ch.n;
  T h = dt / T(double(S));
  T qstar[kMaxDof], arm[kMaxDof], tau[kMaxDof], qdd[kMaxDof];
  for (int j = 0; j < n; ++j) {
    double a = val(action[j]);
    T ac = a > 1.0 ? T(1.0) : (a < -1.0 ? T(-1.0) : action[j]);
    T mid = T(0.5) * (dr.hi[j] + dr.lo[j]);
    T half = T(0.5) * (dr.hi[j] - dr.lo[j]);
    qstar[j] = mid + half * ac;
    arm[j] = h * dr.kd[j] + h * h * dr.kp[j];
  }
  for (int s = 0; s < S; ++s) {
    for (int j = 0; j < n; ++j) tau[j] = dr.kp[j] * (qstar[j] - q[j] - h * qd[j]) - dr.kd[j] * qd[j];
    aba(ch, q, qd, tau, arm, qdd);
    for (int j = 0; j < n; ++j) {
      qd[j] = qd[j] + h * qdd[j];
      q[j] = q[j] + h * qd[j];
      if (q[j] > dr.hi[j]) {
        q[j] = dr.hi[j];
        if (qd[j] > T(0.0)) qd[j] = T(0.0);
      } else if (q[j] < dr.lo[j]) {
        q[j] = dr.lo[j];
        if (qd[j] < T(0.0)) qd[j] = T(0.0);
      }
      if (qdd_log) qdd_log[s * n + j] = qdd[j];
    }
  }
}

template <class T> inline T norm3(const V3<T>& a) {
  using std::sqrt;
  return sqrt(dot(a, a));
}

// Observation of the current state. width = 2*Jmax + 10.
template <class T>
inline void observe(const Chain<T>& ch, int Jmax, const TaskSpec& ts, const EnvGoal<T>& g, const T* q, const T* qd,
                    int progress, T* obs, const Track<T>* tr = nullptr) {
  Pose<T> P;
  forward_kinematics(ch, q, P);
  V3<T> goal = tr ? tr->g : goal_for(ts, g, progress);
  V3<T> d = goal - P.tip;
  for (int j = 0; j < Jmax; ++j) {
    obs[j] = j < ch.n ? q[j] : T(0.0);
    obs[Jmax + j] = j < ch.n ? qd[j] : T(0.0);
  }
  T* o = obs + 2 * Jmax;
  o[0] = P.tip.x; o[1] = P.tip.y; o[2] = P.tip.z;
  o[3] = goal.x;  o[4] = goal.y;  o[5] = goal.z;
  o[6] = d.x;     o[7] = d.y;     o[8] = d.z;
  o[9] = norm3(d);
}

// Whole control step. Returns the done bits; writes reward and obs.
// tr (tracking task only): the env's moving goal, advanced with the draws of
// counter (seed; env, step).
template <class T>
inline uint8_t env_step(const Chain<T>& ch, const Drive<T>& dr, T dt, int S, int Jmax, const TaskSpec& ts,
                        EnvGoal<T>& g, const T* action, T* q, T* qd, int* progress, T* reward, T* obs,
                        T* qdd_log, Track<T>* tr = nullptr, uint64_t seed = 0, uint32_t env = 0,
                        uint64_t step = 0, Rerand<T>* rr = nullptr) {
  physics_step(ch, dr, dt, S, action, q, qd, qdd_log);
  const int n = ch.n;
  Pose<T> P;
  forward_kinematics(ch, q, P);
  int pre = *progress;
  V3<T> goal = tr ? tr->g : goal_for(ts, g, pre);
  *reward = -norm3(P.tip - goal);
  *progress = pre + 1;
  uint8_t done = 0;
  bool finite = true;
  for (int j = 0; j < n; ++j) finite = finite && std::isfinite(val(q[j])) && std::isfinite(val(qd[j]));
  if (!finite) {
    done = kDoneEnded | kDoneNonFinite;
    *reward = T(0.0);
  } else if (ts.ep_len > 0 && *progress >= ts.ep_len) {
    done = kDoneEnded | kDoneTimeout;
  }
  if (done) {
    for (int j = 0; j < n; ++j) {
      q[j] = dr.q0[j];
      qd[j] = T(0.0);
    }
    *progress = 0;
    if (tr) track_reset(ts, *tr, seed, env, step);
    if (rr) {
      rerand_reset(ts, *rr, seed, env, step);
      apply_rerand(ts, *rr, (int)env, g);
    }
  } else if (tr) {
    track_advance(ts, *tr, seed, env, step);
  }
  observe(ch, Jmax, ts, g, q, qd, *progress, obs, tr);
  return done;
}

// One control step of an env made of C chains (paper Sec. IV multi-tool
// reaching): every chain is driven by its own action towards its own goal;
// the env's reward is the sum of the chains' rewards (rho = -1), the episode
// (progress, time-out) is shared, and a non-finite state of any chain ends
// the episode of all of them with reward 0. Returns the done bits; tr (per
// chain, tracking task only) uses Philox env ids lane[c].
template <class T>
inline uint8_t group_step(int C, const Chain<T>* ch, const Drive<T>* dr, T dt, int S, int Jmax, const TaskSpec& ts,
                          const EnvGoal<T>* g, const T* const* action, T* const* q, T* const* qd, int* progress,
                          T* reward, T* const* obs, Track<T>* tr, uint64_t seed, const uint32_t* lane,
                          uint64_t step) {
  const int pre = *progress;
  T rsum = T(0.0);
  bool finite = true;
  for (int c = 0; c < C; ++c) {
    physics_step(ch[c], dr[c], dt, S, action[c], q[c], qd[c], (T*)nullptr);
    Pose<T> P;
    forward_kinematics(ch[c], q[c], P);
    const V3<T> goal = tr ? tr[c].g : goal_for(ts, g[c], pre);
    rsum = rsum - norm3(P.tip - goal);
    for (int j = 0; j < ch[c].n; ++j) finite = finite && std::isfinite(val(q[c][j])) && std::isfinite(val(qd[c][j]));
  }
  *progress = pre + 1;
  uint8_t done = 0;
  if (!finite) {
    done = kDoneEnded | kDoneNonFinite;
    rsum = T(0.0);
  } else if (ts.ep_len > 0 && *progress >= ts.ep_len) {
    done = kDoneEnded | kDoneTimeout;
  }
  for (int c = 0; c < C; ++c) {
    if (done) {
      for (int j = 0; j < ch[c].n; ++j) {
        q[c][j] = dr[c].q0[j];
        qd[c][j] = T(0.0);
      }
      if (tr) track_reset(ts, tr[c], seed, lane[c], step);
    } else if (tr) {
      track_advance(ts, tr[c], seed, lane[c], step);
    }
  }
  if (done) *progress = 0;
  for (int c = 0; c < C; ++c) observe(ch[c], Jmax, ts, g[c], q[c], qd[c], *progress, obs[c], tr ? &tr[c] : nullptr);
  *reward = rsum;
  return done;
}

}  // namespace ora
