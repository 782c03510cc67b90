// Per-lane environment logic around the dynamics: action -> PD target,
// implicit-PD substeps with semi-implicit Euler and hard limits, then
// tool-tip kinematics, reward, episode bookkeeping, auto-reset and the
// observation (paper Sec. III "Simulation Setup", "Action Space",
// "Observation Space", "Policy learning and control"; Sec. IV target
// reaching and path following rewards).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dyn.hpp"
#include "rng.hpp"

namespace sgk {

enum { TASK_REACH = 0, TASK_PATH = 1, TASK_TRACK = 2 };
// Kernel variants: per-env joint counts (M_GEN); every env with exactly the
// kernel's J joints, so the per-joint guards fold away (M_UNI); per-env
// joint counts with revolute and prismatic joints (M_PRI).
enum { M_GEN = 0, M_UNI = 1, M_PRI = 2 };
enum { DONE_ENDED = 1, DONE_TIMEOUT = 2, DONE_NONFINITE = 4 };

template <typename T> struct EnvDev {
  int N, J, S, task, K, dwell, ep_len;
  int chains;         // consecutive lanes (chains) per env: 1, 2 or 4
  T dt, h, g[3];
  const T* par;       // [P_NFIELDS][J][N]
  const T* tip;       // [3][N]
  const T* tip0;      // [3][N] tool tip at q0 (the reset pose)
  const int* nd;      // [N]
  const T* target;    // [3][N]
  const T* wp;        // [K][3][N]
  const int* prog0;   // [N]
  T* q;               // [J][N]
  T* qd;              // [J][N]
  int* prog;          // [N]
  // tracking task: moving goal [9][N] = goal, goal velocity, episode centre;
  // random walk sigma, offset box, reset spread and nominal centre
  T* gs;
  T trk_sigma, trk_offset, trk_reset_std, trk_c[3];
  // per-episode re-randomisation (reach: gs [3][N] = the episode's target;
  // path: gs [1][N] = the index of its waypoint set of nbank sets)
  int rerand, nbank;
  T rc[3], rhalf;
  uint64_t seed;      // noise key
  uint64_t* rng;      // device noise counter: control steps drawn so far
  unsigned* tick;     // blocks of the current launch that have read *rng
  uint32_t rng_add;   // this launch advances *rng by rng_add (0: leaves it)
};

// The noise counter at the start of this launch (read by every thread that
// needs it, before advance_counter runs in its block).
template <typename T> __device__ __forceinline__ uint64_t read_counter(const EnvDev<T>& E) {
  return __atomic_load_n(E.rng, __ATOMIC_RELAXED);
}

// Waits until a value loaded from memory has returned (its register is an
// operand here, so the compiler waits for the load before this point).
__device__ __forceinline__ void settle(uint64_t v) {
  asm volatile("" ::"v"((uint32_t)v), "v"((uint32_t)(v >> 32)));
}

// With E.rng_add != 0, advances the counter by rng_add so that the next
// launch (or the next replay of a captured graph) draws fresh noise. One
// thread per block calls it at the block's end. If the launch read the
// counter (readers: v = the value this block read, and every thread of the
// block has read it), each block takes a ticket once its read has returned
// and the last block stores v + rng_add; the counter and ticket are written
// by plain stores that the next launch sees. If no block read it, block 0
// alone adds rng_add.
template <typename T>
__device__ __forceinline__ void advance_counter(const EnvDev<T>& E, uint64_t v, bool readers) {
  if (!E.rng_add) return;
  if (!readers) {
    if (blockIdx.x == 0) *E.rng = *E.rng + E.rng_add;
    return;
  }
  settle(v);  // this wave's read has returned before the ticket is taken
  const unsigned nb = gridDim.x * gridDim.y * gridDim.z;
  if (atomicAdd(E.tick, 1u) == nb - 1) {
    *E.rng = v + E.rng_add;
    *E.tick = 0u;
  }
}

// Link parameters of env e into registers (joints < n).
template <typename T, int J, bool PR>
__device__ __forceinline__ void load_chain(const EnvDev<T>& E, int e, int n, RegPar<T, J, PR>& rp) {
#pragma unroll
  for (int j = 0; j < J; ++j) {
    if (j < n) load_joint(E.par, E.J, E.N, j, e, rp.P[j]);
  }
}

// Stage the link parameters of a 64-env block into LDS [P_NSTAGE][J][64]
// (joints >= n zero). Every lane of the block calls it; the caller
// synchronizes before use.
template <typename T, int J>
__device__ __forceinline__ void stage_chain(const EnvDev<T>& E, int e, int n, int lane, T* sp) {
  for (int f = 0; f < P_NSTAGE; ++f)
#pragma unroll
    for (int j = 0; j < J; ++j)
      sp[(f * J + j) * 64 + lane] = (j < n) ? E.par[((size_t)f * E.J + j) * E.N + e] : T(0);
}

// The same staging for a block whose 64 envs are contiguous (e0 .. e0 + 63):
// every [field][joint] row of the block is 64 consecutive values of the
// parameter block, copied by 16 threads as 16-byte pieces (FP32), NT / 16
// rows at a time by the block's NT threads (tid = 0 .. NT-1); values of
// envs past the last one, and of joints past max_dof, zero. The parameter
// block holds zeros for joints >= an env's n_dof, as stage_chain writes.
template <typename T, int J, int NT = 64>
__device__ __forceinline__ void stage_block(const EnvDev<T>& E, int e0, int tid, T* sp) {
  if constexpr (sizeof(T) != 4) {
    static_assert(NT == 64, "FP64 staging runs one lane per env");
    stage_chain<T, J>(E, e0 + tid, e0 + tid < E.N ? J : 0, tid, sp);
  } else {
    constexpr int rows = P_NSTAGE * J;
    constexpr int kRows = NT / 16;                     // rows per pass
    constexpr int kIter = (rows + kRows - 1) / kRows;  // passes
    const int sub = tid >> 4, c = (tid & 15) * 4;
    const bool full = (E.N & 3) == 0 && e0 + 64 <= E.N;
    if (full) {
      // every row whole: all of this thread's loads issued before any LDS
      // store (a fixed trip count the compiler unrolls)
      float4 v[kIter];
#pragma unroll
      for (int k = 0; k < kIter; ++k) {
        const int r = kRows * k + sub;
        const int f = r / J, j = r % J;
        v[k] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (r < rows && j < E.J) v[k] = *reinterpret_cast<const float4*>(E.par + ((size_t)f * E.J + j) * E.N + e0 + c);
      }
#pragma unroll
      for (int k = 0; k < kIter; ++k) {
        const int r = kRows * k + sub;
        if (r < rows) *reinterpret_cast<float4*>(sp + r * 64 + c) = v[k];
      }
      return;
    }
    for (int r = sub; r < rows; r += kRows) {
      const int f = r / J, j = r % J;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (j < E.J) {
        const T* src = E.par + ((size_t)f * E.J + j) * E.N + e0 + c;
        v.x = e0 + c < E.N ? src[0] : 0.f;
        v.y = e0 + c + 1 < E.N ? src[1] : 0.f;
        v.z = e0 + c + 2 < E.N ? src[2] : 0.f;
        v.w = e0 + c + 3 < E.N ? src[3] : 0.f;
      }
      *reinterpret_cast<float4*>(sp + r * 64 + c) = v;
    }
  }
}

// ---- per-block parameter sources ----------------------------------------
constexpr int kBlk = 64;

template <typename T, int J> constexpr size_t par_lds_bytes() { return sizeof(T) * P_NSTAGE * J * kBlk; }
// LDS staging when the block's parameters fit comfortably, else registers.
template <typename T, int J> constexpr bool use_lds() { return par_lds_bytes<T, J>() <= 96 * 1024; }

// Parameter source for env e of this block: LDS-staged (after a barrier) or
// register-held. Every lane of the block must call it (barrier inside).
template <typename T, int J, bool LDS, bool PR> struct ParOf;
template <typename T, int J, bool PR> struct ParOf<T, J, true, PR> {
  using type = LdsPar<T, J, PR>;
  static __device__ __forceinline__ type make(const EnvDev<T>& E, int e, int n, bool active, T* sp) {
    __syncthreads();  // the block may be re-staging for its next tile
    stage_chain<T, J>(E, e, active ? n : 0, threadIdx.x, sp);
    __syncthreads();
    return type{sp, (int)threadIdx.x};
  }
  // blocks of 64 contiguous envs: e = 64 blockIdx.x + threadIdx.x
  static __device__ __forceinline__ type make_contiguous(const EnvDev<T>& E, T* sp) {
    __syncthreads();
    stage_block<T, J>(E, (int)blockIdx.x * kBlk, threadIdx.x, sp);
    __syncthreads();
    return type{sp, (int)threadIdx.x};
  }
};
template <typename T, int J, bool PR> struct ParOf<T, J, false, PR> {
  using type = RegPar<T, J, PR>;
  static __device__ __forceinline__ type make(const EnvDev<T>& E, int e, int n, bool active, T*) {
    type r;
    if (active) load_chain<T, J>(E, e, n, r);
    return r;
  }
  static __device__ __forceinline__ type make_contiguous(const EnvDev<T>& E, T*) {
    const int e = (int)blockIdx.x * kBlk + threadIdx.x;
    const int n = e < E.N ? E.nd[e] : 0;
    type r;
    if (e < E.N) load_chain<T, J>(E, e, n, r);
    return r;
  }
};

template <typename T, int J>
__device__ __forceinline__ void load_state(const EnvDev<T>& E, int e, int n, T (&q)[J], T (&qd)[J]) {
#pragma unroll
  for (int j = 0; j < J; ++j) {
    q[j] = j < n ? E.q[(size_t)j * E.N + e] : T(0);
    qd[j] = j < n ? E.qd[(size_t)j * E.N + e] : T(0);
  }
}

template <typename T> __device__ __forceinline__ T clamp1(T a) { return a > T(1) ? T(1) : (a < T(-1) ? T(-1) : a); }

// S substeps of the implicit-PD step with the action held (zero-order hold).
// TEAM: the solve is shared with the workgroup's helper waves (aba_lwa_team;
// the helpers run physics_help meanwhile).
template <typename T, int J, class PS, bool TEAM = false>
__device__ __forceinline__ void physics(const EnvDev<T>& E, PS& ps, int n, const T (&act)[J], T (&q)[J],
                                        T (&qd)[J], const TeamLds& team = TeamLds{}) {
  const T h = E.h;
  T qs[J], arm[J], tau[J], qdd[J];
  ps.fence();
#pragma unroll
  for (int j = 0; j < J; ++j) {
    if (j < n) {
      const Jp<T> p = ps.get(j);
      const T mid = T(0.5) * (p.hi + p.lo), half = T(0.5) * (p.hi - p.lo);
      qs[j] = mid + half * clamp1(act[j]);
      arm[j] = h * p.kd + h * h * p.kp;
    } else {
      qs[j] = T(0);
      arm[j] = T(0);
    }
  }
  for (int s = 0; s < E.S; ++s) {
    // the helpers start on the published state while the torques are formed
    if constexpr (TEAM) team_publish<J>(team, q, qd);
    ps.fence();
#pragma unroll
    for (int j = 0; j < J; ++j) {
      if (j < n) {
        const Jp<T> p = ps.get(j);
        tau[j] = p.kp * (qs[j] - q[j] - h * qd[j]) - p.kd * qd[j];
      } else {
        tau[j] = T(0);
      }
    }
    if constexpr (TEAM) aba_lwa_team<J>(ps, n, q, qd, tau, arm, E.g, qdd, team);
    else aba_lwa<T, J>(ps, n, q, qd, tau, arm, E.g, qdd);
    ps.fence();
#pragma unroll
    for (int j = 0; j < J; ++j) {
      if (j < n) {
        const Jp<T> p = ps.get(j);
        qd[j] = qd[j] + h * qdd[j];
        q[j] = q[j] + h * qd[j];
        if (q[j] > p.hi) {
          q[j] = p.hi;
          if (qd[j] > T(0)) qd[j] = T(0);
        } else if (q[j] < p.lo) {
          q[j] = p.lo;
          if (qd[j] < T(0)) qd[j] = T(0);
        }
      }
    }
  }
}

// A helper wave's side of a team physics() call: one team solve per substep;
// after_first() runs once the first substep's links are handed back, while
// wave 0 runs that substep's inward and outward passes.
template <int J, class PS, class F>
__device__ __forceinline__ void physics_help(const EnvDev<float>& E, PS& ps, int n, const TeamLds& team,
                                             F&& after_first) {
  for (int s = 0; s < E.S; ++s) {
    aba_team_help<J>(ps, n, team);
    if (s == 0) after_first();
  }
}
template <int J, class PS>
__device__ __forceinline__ void physics_help(const EnvDev<float>& E, PS& ps, int n, const TeamLds& team) {
  physics_help<J>(E, ps, n, team, [] {});
}

template <typename T>
__device__ __forceinline__ void goal_of(const EnvDev<T>& E, int e, int progress, T* g) {
  if (E.task == TASK_TRACK) {
    g[0] = E.gs[e];
    g[1] = E.gs[E.N + e];
    g[2] = E.gs[2 * E.N + e];
  } else if (E.task == TASK_REACH) {
    const T* t = E.rerand ? E.gs : E.target;
    g[0] = t[e];
    g[1] = t[E.N + e];
    g[2] = t[2 * E.N + e];
  } else {
    int k = progress / E.dwell;
    k = k > E.K - 1 ? E.K - 1 : k;
    const int bank = E.rerand ? (int)E.gs[e] : 0;
    const T* w = E.wp + ((size_t)bank * E.K + k) * 3 * E.N;
    g[0] = w[e];
    g[1] = w[E.N + e];
    g[2] = w[2 * E.N + e];
  }
}

template <typename T, int J>
__device__ __forceinline__ void write_obs(const EnvDev<T>& E, int e, int n, const T (&q)[J], const T (&qd)[J],
                                          const T* tip, const T* g, T* __restrict__ obs) {
  const size_t N = E.N;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    if (j < E.J) {
      obs[(size_t)j * N + e] = j < n ? q[j] : T(0);
      obs[(size_t)(E.J + j) * N + e] = j < n ? qd[j] : T(0);
    }
  }
  // a kernel specialised for fewer joints than the context's max_dof (DOF-
  // class tiles) still owns the padded rows
  for (int j = J; j < E.J; ++j) {
    obs[(size_t)j * N + e] = T(0);
    obs[(size_t)(E.J + j) * N + e] = T(0);
  }
  T* o = obs + (size_t)(2 * E.J) * N + e;
  const T dx = g[0] - tip[0], dy = g[1] - tip[1], dz = g[2] - tip[2];
  o[0] = tip[0]; o[N] = tip[1]; o[2 * N] = tip[2];
  o[3 * N] = g[0]; o[4 * N] = g[1]; o[5 * N] = g[2];
  o[6 * N] = dx; o[7 * N] = dy; o[8 * N] = dz;
  o[9 * N] = rsq(dx * dx + dy * dy + dz * dz);
}

template <typename T> __device__ __forceinline__ bool finite_(T x) { return isfinite(x); }

// Observation row in registers (width 2*E.J + 10, entries beyond zero-padded
// up to the caller's array size).
template <typename T, int J, int WMAX>
__device__ __forceinline__ void obs_regs(const EnvDev<T>& E, int n, const T (&q)[J], const T (&qd)[J], const T* tip,
                                         const T* g, T (&x)[WMAX]) {
#pragma unroll
  for (int k = 0; k < WMAX; ++k) x[k] = T(0);
#pragma unroll
  for (int j = 0; j < J; ++j) {
    if (j < E.J) {
      x[j] = j < n ? q[j] : T(0);
      x[E.J + j] = j < n ? qd[j] : T(0);
    }
  }
  const T dx = g[0] - tip[0], dy = g[1] - tip[1], dz = g[2] - tip[2];
  const int b = 2 * E.J;
  x[b + 0] = tip[0]; x[b + 1] = tip[1]; x[b + 2] = tip[2];
  x[b + 3] = g[0];   x[b + 4] = g[1];   x[b + 5] = g[2];
  x[b + 6] = dx;     x[b + 7] = dy;     x[b + 8] = dz;
  x[b + 9] = rsq(dx * dx + dy * dy + dz * dz);
}

// Tracking task (paper Sec. IV "Active Tracking"): after a step that did not
// end the episode the goal moves by its velocity, is held inside the offset
// box around the episode centre (dropping the outward velocity component),
// and the velocity takes a random increment; a new episode draws a new
// centre and starts the goal on it at rest.
template <typename T>
__device__ __forceinline__ void track_update(const EnvDev<T>& E, int e, bool reset, uint64_t step) {
  const size_t N = E.N;
  T* gs = E.gs + e;
  float n4[4];
  if (reset) {
    normals4(E.seed, (uint32_t)e, step, RNG_BLOCK_GOAL_RESET, n4);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const T c = E.trk_c[k] + E.trk_reset_std * (T)n4[k];
      gs[k * N] = c;
      gs[(3 + k) * N] = T(0);
      gs[(6 + k) * N] = c;
    }
    return;
  }
  normals4(E.seed, (uint32_t)e, step, RNG_BLOCK_GOAL_ACCEL, n4);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T g = gs[k * N], gd = gs[(3 + k) * N];
    const T c = gs[(6 + k) * N];
    g = g + gd;
    const T hi = c + E.trk_offset, lo = c - E.trk_offset;
    if (g > hi) {
      g = hi;
      if (gd > T(0)) gd = T(0);
    } else if (g < lo) {
      g = lo;
      if (gd < T(0)) gd = T(0);
    }
    gs[k * N] = g;
    gs[(3 + k) * N] = gd + E.trk_sigma * (T)n4[k];
  }
}

// Per-episode re-randomisation at a reset: the next episode's goal from
// Philox block RNG_BLOCK_RERAND of (env, step). Reach: target_k = centre_k +
// half (2 u_k - 1) with u_k the 24-bit uniform of word k; path: the
// waypoint set (word 0 >> 8) nbank / 2^24 in integer arithmetic.
template <typename T> __device__ __forceinline__ void rerand_draw(const EnvDev<T>& E, int e, uint64_t step) {
  const U4 r = philox10(U4{(uint32_t)e, (uint32_t)step, (uint32_t)(step >> 32), (uint32_t)RNG_BLOCK_RERAND},
                        (uint32_t)E.seed, (uint32_t)(E.seed >> 32));
  if (E.task == TASK_REACH) {
    const uint32_t w[3] = {r.x, r.y, r.z};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const T u = ((T)(w[k] >> 8) + T(0.5)) * (T(1) / T(16777216));
      E.gs[(size_t)k * E.N + e] = E.rc[k] + E.rhalf * (T(2) * u - T(1));
    }
  } else {
    E.gs[e] = (T)(int)(((uint64_t)(r.x >> 8) * (uint64_t)E.nbank) >> 24);
  }
}

// After the physics: reward on the post-step tip against the goal active
// during the step, progress, time-out or non-finite reset, the tracking
// goal's update, observation of the post-reset state. step = this control
// step's counter (noise of the tracking task). Returns the done bits;
// *reward receives the reward.
template <typename T, int J, class PS>
__device__ __forceinline__ uint8_t post_step(const EnvDev<T>& E, int e, int n, PS& ps, T (&q)[J], T (&qd)[J],
                                             int& prog, T* reward, T* __restrict__ obs, T* tip_out = nullptr,
                                             T* goal_out = nullptr, uint64_t step = 0) {
  const T tipl[3] = {E.tip[e], E.tip[E.N + e], E.tip[2 * E.N + e]};
  T tip[3], g[3];
  // the joint angles' sin and cos from the hardware in FP32 (about 1e-6 m
  // on the tip, far inside the reward's and observation's rounding budget)
  tip_fk<T, J, PS, true>(ps, n, q, tipl, tip);
  goal_of(E, e, prog, g);
  const T dx = tip[0] - g[0], dy = tip[1] - g[1], dz = tip[2] - g[2];
  T r = -rsq(dx * dx + dy * dy + dz * dz);
  prog = prog + 1;
  bool fin = true;
#pragma unroll
  for (int j = 0; j < J; ++j)
    if (j < n) fin = fin && finite_(q[j]) && finite_(qd[j]);
  if (E.chains > 1) {
    // an env of several chains (consecutive lanes of one wave, all active):
    // the reward is their sum and any non-finite chain ends the episode of all
    int bad = fin ? 0 : 1;
    for (int m = 1; m < E.chains; m <<= 1) {
      r += __shfl_xor(r, m, 64);
      bad |= __shfl_xor(bad, m, 64);
    }
    fin = bad == 0;
  }
  uint8_t done = 0;
  if (!fin) {
    done = DONE_ENDED | DONE_NONFINITE;
    r = T(0);
  } else if (E.ep_len > 0 && prog >= E.ep_len) {
    done = DONE_ENDED | DONE_TIMEOUT;
  }
  if (done) {
#pragma unroll
    for (int j = 0; j < J; ++j) {
      if (j < n) {
        q[j] = E.par[((size_t)P_Q0 * E.J + j) * E.N + e];
        qd[j] = T(0);
      }
    }
    prog = 0;
    // the reset pose's tip, computed once at create
    tip[0] = E.tip0[e];
    tip[1] = E.tip0[E.N + e];
    tip[2] = E.tip0[2 * E.N + e];
  }
  if (E.task == TASK_TRACK) track_update(E, e, done != 0, step);
  if (E.rerand && done) rerand_draw(E, e, step);
  goal_of(E, e, prog, g);
  if (obs) write_obs<T, J>(E, e, n, q, qd, tip, g, obs);
  if (tip_out) { tip_out[0] = tip[0]; tip_out[1] = tip[1]; tip_out[2] = tip[2]; }
  if (goal_out) { goal_out[0] = g[0]; goal_out[1] = g[1]; goal_out[2] = g[2]; }
  *reward = r;
  return done;
}

template <typename T, int J>
__device__ __forceinline__ void store_state(const EnvDev<T>& E, int e, int n, const T (&q)[J], const T (&qd)[J],
                                            int prog) {
#pragma unroll
  for (int j = 0; j < J; ++j) {
    if (j < n) {
      E.q[(size_t)j * E.N + e] = q[j];
      E.qd[(size_t)j * E.N + e] = qd[j];
    }
  }
  E.prog[e] = prog;
}

}  // namespace sgk
