// Environment-step kernels: one environment per lane, chain state in VGPRs,
// the block's link parameters staged in LDS ([P_NSTAGE][J][64]) and read
// per pass, structure-of-arrays global layout so each per-joint field is one
// coalesced 64-lane access. The kernel variant M (M_GEN, M_UNI, M_PRI) picks
// per-env joint counts, exactly J joints, or chains with prismatic joints.
#include <mutex>
#include <set>
#include <utility>

#include "internal.hpp"

namespace sgk {

hipError_t lds_limit(const void* fn, size_t bytes) {
  if (bytes <= 64 * 1024) return hipSuccess;
  static std::mutex mu;
  static std::set<std::pair<int, const void*>> done;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  if (done.count({dev, fn})) return hipSuccess;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess) done.insert({dev, fn});
  return e;
}

int dof_bucket(int J) {
  if (J <= 1) return 1;
  if (J <= 2) return 2;
  if (J <= 4) return 4;
  if (J <= 7) return 7;
  if (J <= 9) return 9;
  return 16;
}

#define SG_PAR_SETUP                                                                 \
  extern __shared__ __align__(16) unsigned char smem_raw[];                          \
  T* sp = reinterpret_cast<T*>(smem_raw);                                            \
  const int e = blockIdx.x * kBlk + threadIdx.x;                                     \
  const bool active = e < E.N;                                                       \
  const int n = M == M_UNI ? J : (active ? E.nd[e] : 0);                            \
  auto ps = ParOf<T, J, use_lds<T, J>(), M == M_PRI>::make(E, e, n, active, sp);     \
  if (!active) return;

// One control step of env e (inactive lanes only help stage parameters).
// CONTIG: the block's envs are 64 blockIdx.x .. + 63: the parameters are
// staged as contiguous rows, and (FP32) the state and action loads are
// issued before the staging, overlapping it.
template <typename T, int J, int M, bool CONTIG = false>
__device__ __forceinline__ void step_body(const EnvDev<T>& E, int e, bool active, T* sp, const T* __restrict__ act,
                                          T* __restrict__ obs, T* __restrict__ rew, uint8_t* __restrict__ done,
                                          uint64_t step) {
  const int n = M == M_UNI ? J : (active ? E.nd[e] : 0);
  // (FP64 keeps the later loads: its state held across the staging spills)
  constexpr bool EARLY = CONTIG && sizeof(T) == 4;
  T q[J], qd[J], a[J];
  if (EARLY && active) {
    load_state<T, J>(E, e, n, q, qd);
#pragma unroll
    for (int j = 0; j < J; ++j) a[j] = j < n ? act[(size_t)j * E.N + e] : T(0);
  }
  using Src = ParOf<T, J, use_lds<T, J>(), M == M_PRI>;
  auto ps = CONTIG ? Src::make_contiguous(E, sp) : Src::make(E, e, n, active, sp);
  if (!active) return;
  if (!EARLY) {
    load_state<T, J>(E, e, n, q, qd);
#pragma unroll
    for (int j = 0; j < J; ++j) a[j] = j < n ? act[(size_t)j * E.N + e] : T(0);
  }
  physics<T, J>(E, ps, n, a, q, qd);
  int prog = E.prog[e];
  T r;
  const uint8_t d = post_step<T, J>(E, e, n, ps, q, qd, prog, &r, obs, nullptr, nullptr, step);
  store_state<T, J>(E, e, n, q, qd, prog);
  rew[e] = r;
  done[e] = d;
}

template <typename T, int J, int M>
__global__ void __launch_bounds__(kBlk) k_step(EnvDev<T> E, const T* __restrict__ act, T* __restrict__ obs,
                                               T* __restrict__ rew, uint8_t* __restrict__ done) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int e = blockIdx.x * kBlk + threadIdx.x;
  // only the tracking task and re-randomised goals draw noise in the step
  const bool reads = E.task == TASK_TRACK || E.rerand;
  const uint64_t step = reads ? read_counter(E) : 0;
  step_body<T, J, M, true>(E, e, e < E.N, reinterpret_cast<T*>(smem_raw), act, obs, rew, done, step);
  // one wave per block: every lane read the counter above
  if (threadIdx.x == 0) advance_counter(E, step, reads);
}

// One control step with a wave team (FP32; kTeam waves per 64 contiguous
// envs): the four waves stage the block's parameters together, wave 0 runs
// the step with every substep's solve shared as in the fused rollout
// (aba_lwa_team), the other waves run their side of each solve. Wave 0 runs
// the physics for all of its lanes (lanes past N on zero parameters, storing
// nothing), so every wave meets every barrier.
__host__ __device__ constexpr size_t team_state_bytes(int J) { return (size_t)team_state_slots(J) * 64 * 16; }
template <int J> constexpr size_t team_step_lds_bytes() {
  return par_lds_bytes<float, J>() + team_state_bytes(J) + team_lds_bytes(J);
}
static_assert(team_step_lds_bytes<9>() <= 160 * 1024, "the 9-joint team step fits the LDS");

template <int J, int M>
__global__ void __launch_bounds__(kBlk * kTeam) k_step_team(EnvDev<float> E, const float* __restrict__ act,
                                                            float* __restrict__ obs, float* __restrict__ rew,
                                                            uint8_t* __restrict__ done) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float* sp = reinterpret_cast<float*>(smem_raw);
  const TeamLds team{reinterpret_cast<float4*>(smem_raw + par_lds_bytes<float, J>()),
                     reinterpret_cast<float4*>(smem_raw + par_lds_bytes<float, J>() + team_state_bytes(J)),
                     (int)(threadIdx.x >> 6), (int)(threadIdx.x & (kBlk - 1))};
  const int e = blockIdx.x * kBlk + team.lane;
  const bool active = e < E.N;
  const int n = M == M_UNI ? J : (active ? E.nd[e] : 0);
  // only the tracking task and re-randomised goals draw noise in the step
  const bool reads = E.task == TASK_TRACK || E.rerand;
  const uint64_t step = reads ? read_counter(E) : 0;
  float q[J], qd[J], a[J];
#pragma unroll
  for (int j = 0; j < J; ++j) { q[j] = 0.f; qd[j] = 0.f; a[j] = 0.f; }
  if (team.wave == 0 && active) {
    // issued before the staging, overlapping it
    load_state<float, J>(E, e, n, q, qd);
#pragma unroll
    for (int j = 0; j < J; ++j) a[j] = j < n ? act[(size_t)j * E.N + e] : 0.f;
  }
  stage_block<float, J, kBlk * kTeam>(E, (int)blockIdx.x * kBlk, threadIdx.x, sp);
  __syncthreads();
  LdsPar<float, J, M == M_PRI> ps{sp, team.lane};
  if (team.wave == 0) {
    physics<float, J, LdsPar<float, J, M == M_PRI>, true>(E, ps, n, a, q, qd, team);
    if (active) {
      int prog = E.prog[e];
      float r;
      const uint8_t d = post_step<float, J>(E, e, n, ps, q, qd, prog, &r, obs, nullptr, nullptr, step);
      store_state<float, J>(E, e, n, q, qd, prog);
      rew[e] = r;
      done[e] = d;
    }
  } else {
    physics_help<J>(E, ps, n, team);
  }
  // every wave read the counter before the staging barrier
  if (threadIdx.x == 0) advance_counter(E, step, reads);
}

// Uneven batches: envs bucketed by DOF class into 64-slot tiles, so every
// block is class-homogeneous and runs the class's specialised code (exact
// joint count where instantiated, else the next size with per-joint guards).
// Tiles [tile0, tile0 + ntiles) are walked with a grid-stride loop, so one
// launch can cover all classes (fused), one class (per-class launches), or
// all tiles with fewer resident blocks (persistent).
template <typename T, int JB>
__device__ __forceinline__ void step_tile(const EnvDev<T>& E, int nd, int e, T* sp, const T* act, T* obs, T* rew,
                                          uint8_t* done, uint64_t st) {
  const bool active = e >= 0;
  if (nd == 1) step_body<T, 1, M_UNI>(E, e, active, sp, act, obs, rew, done, st);
  else if (nd == 2) step_body<T, 2, M_UNI>(E, e, active, sp, act, obs, rew, done, st);
  else if (nd == 4) step_body<T, 4, M_UNI>(E, e, active, sp, act, obs, rew, done, st);
  else if (nd == 3) step_body<T, 4, M_GEN>(E, e, active, sp, act, obs, rew, done, st);
  else if (JB >= 6 && nd == 6) step_body<T, (JB >= 6 ? 6 : 4), M_UNI>(E, e, active, sp, act, obs, rew, done, st);
  else if (JB >= 6 && nd == 5) step_body<T, (JB >= 6 ? 6 : 4), M_GEN>(E, e, active, sp, act, obs, rew, done, st);
  else if (JB >= 7 && nd == 7) step_body<T, (JB >= 7 ? 7 : 4), M_UNI>(E, e, active, sp, act, obs, rew, done, st);
  else if (JB >= 9 && nd == 9) step_body<T, (JB >= 9 ? 9 : 4), M_UNI>(E, e, active, sp, act, obs, rew, done, st);
  else if (JB >= 9 && nd == 8) step_body<T, (JB >= 9 ? 9 : 4), M_GEN>(E, e, active, sp, act, obs, rew, done, st);
  else step_body<T, JB, M_GEN>(E, e, active, sp, act, obs, rew, done, st);
}

template <typename T, int JB>
__global__ void __launch_bounds__(kBlk) k_step_tiles(EnvDev<T> E, const int* __restrict__ slot_env,
                                                     const int* __restrict__ tile_dof, int tile0, int ntiles,
                                                     const T* __restrict__ act, T* __restrict__ obs,
                                                     T* __restrict__ rew, uint8_t* __restrict__ done) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sp = reinterpret_cast<T*>(smem_raw);
  const bool reads = E.task == TASK_TRACK || E.rerand;
  const uint64_t st = reads ? read_counter(E) : 0;
  for (int t = tile0 + blockIdx.x; t < tile0 + ntiles; t += gridDim.x) {
    const int e = slot_env[(size_t)t * kBlk + threadIdx.x];
    step_tile<T, JB>(E, tile_dof[t], e, sp, act, obs, rew, done, st);
  }
  if (threadIdx.x == 0) advance_counter(E, st, reads);
}

template <typename T, int J, int M>
__global__ void __launch_bounds__(kBlk) k_observe(EnvDev<T> E, T* __restrict__ obs) {
  SG_PAR_SETUP
  T q[J], qd[J];
  load_state<T, J>(E, e, n, q, qd);
  const T tipl[3] = {E.tip[e], E.tip[E.N + e], E.tip[2 * E.N + e]};
  T tip[3], g[3];
  tip_fk<T, J>(ps, n, q, tipl, tip);
  goal_of(E, e, E.prog[e], g);
  write_obs<T, J>(E, e, n, q, qd, tip, g, obs);
}

template <typename T, int J, int M>
__global__ void __launch_bounds__(kBlk) k_fd(EnvDev<T> E, const T* __restrict__ qin, const T* __restrict__ qdin,
                                             const T* __restrict__ tauin, int arm_mode, T* __restrict__ qddout) {
  SG_PAR_SETUP
  T q[J], qd[J], tau[J], arm[J], qdd[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const size_t i = (size_t)j * E.N + e;
    q[j] = j < n ? qin[i] : T(0);
    qd[j] = j < n ? qdin[i] : T(0);
    tau[j] = j < n ? tauin[i] : T(0);
    if (j < n && arm_mode == SG_ARM_DRIVE) {
      const Jp<T> p = ps.get(j);
      arm[j] = E.h * p.kd + E.h * E.h * p.kp;
    } else {
      arm[j] = T(0);
    }
  }
  aba_lwa<T, J>(ps, n, q, qd, tau, arm, E.g, qdd);
#pragma unroll
  for (int j = 0; j < J; ++j)
    if (j < E.J) qddout[(size_t)j * E.N + e] = j < n ? qdd[j] : T(0);
}

template <typename T, int J, int M>
__global__ void __launch_bounds__(kBlk) k_id(EnvDev<T> E, const T* __restrict__ qin, const T* __restrict__ qdin,
                                             const T* __restrict__ qddin, T* __restrict__ tauout) {
  SG_PAR_SETUP
  T q[J], qd[J], qdd[J], tau[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const size_t i = (size_t)j * E.N + e;
    q[j] = j < n ? qin[i] : T(0);
    qd[j] = j < n ? qdin[i] : T(0);
    qdd[j] = j < n ? qddin[i] : T(0);
  }
  rnea<T, J>(ps, n, q, qd, qdd, E.g, tau);
#pragma unroll
  for (int j = 0; j < J; ++j)
    if (j < E.J) tauout[(size_t)j * E.N + e] = j < n ? tau[j] : T(0);
}

template <typename T, int J, int M>
__global__ void __launch_bounds__(kBlk) k_tip(EnvDev<T> E, const T* __restrict__ qin, T* __restrict__ out) {
  SG_PAR_SETUP
  T q[J];
#pragma unroll
  for (int j = 0; j < J; ++j) q[j] = j < n ? qin[(size_t)j * E.N + e] : T(0);
  const T tipl[3] = {E.tip[e], E.tip[E.N + e], E.tip[2 * E.N + e]};
  T tip[3];
  tip_fk<T, J>(ps, n, q, tipl, tip);
  out[e] = tip[0];
  out[E.N + e] = tip[1];
  out[2 * E.N + e] = tip[2];
}

__global__ void k_set_counter(uint64_t* ctr, uint64_t v) {
  if (threadIdx.x == 0) *ctr = v;
}

hipError_t launch_set_counter(const sg_ctx* c, uint64_t value) {
  k_set_counter<<<1, 64, 0, c->stream>>>(c->rng_dev, value);
  return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(256) k_reset(EnvDev<T> E) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= E.N) return;
  for (int j = 0; j < E.J; ++j) {
    const size_t i = (size_t)j * E.N + e;
    E.q[i] = E.par[(size_t)P_Q0 * E.J * E.N + i];
    E.qd[i] = T(0);
  }
  E.prog[e] = E.prog0[e];
}

// Launch with the block's dynamic LDS (the kernel's LDS limit raised above
// the 64 KB default where needed).
template <typename T, int J, typename K, typename... Args>
static hipError_t launch_par(K kernel, const sg_ctx* c, Args... args) {
  constexpr size_t lds = use_lds<T, J>() ? par_lds_bytes<T, J>() : 0;
  hipError_t e = lds_limit((const void*)kernel, lds);
  if (e != hipSuccess) return e;
  kernel<<<dim3((c->N + kBlk - 1) / kBlk), kBlk, lds, c->stream>>>(args...);
  return hipGetLastError();
}

#define SG_DISPATCH(KERNEL, T_, ...)                                                               \
  do {                                                                                             \
    const bool uni = c->uniform;                                                                   \
    if (c->prismatic) {                                                                            \
      switch (dof_bucket(c->J)) {                                                                  \
        case 1: case 2: case 4: return launch_par<T_, 4>(KERNEL<T_, 4, M_PRI>, c, __VA_ARGS__);    \
        case 7: return launch_par<T_, 7>(KERNEL<T_, 7, M_PRI>, c, __VA_ARGS__);                    \
        case 9: return launch_par<T_, 9>(KERNEL<T_, 9, M_PRI>, c, __VA_ARGS__);                    \
        default: return launch_par<T_, 16>(KERNEL<T_, 16, M_PRI>, c, __VA_ARGS__);                 \
      }                                                                                            \
    }                                                                                              \
    switch (dof_bucket(c->J)) {                                                                    \
      case 1: return launch_par<T_, 1>(KERNEL<T_, 1, M_UNI>, c, __VA_ARGS__);                      \
      case 2: return uni ? launch_par<T_, 2>(KERNEL<T_, 2, M_UNI>, c, __VA_ARGS__)                 \
                         : launch_par<T_, 2>(KERNEL<T_, 2, M_GEN>, c, __VA_ARGS__);                \
      case 4: return uni ? launch_par<T_, 4>(KERNEL<T_, 4, M_UNI>, c, __VA_ARGS__)                 \
                         : launch_par<T_, 4>(KERNEL<T_, 4, M_GEN>, c, __VA_ARGS__);                \
      case 7: return uni ? launch_par<T_, 7>(KERNEL<T_, 7, M_UNI>, c, __VA_ARGS__)                 \
                         : launch_par<T_, 7>(KERNEL<T_, 7, M_GEN>, c, __VA_ARGS__);                \
      case 9: return uni ? launch_par<T_, 9>(KERNEL<T_, 9, M_UNI>, c, __VA_ARGS__)                 \
                         : launch_par<T_, 9>(KERNEL<T_, 9, M_GEN>, c, __VA_ARGS__);                \
      default: return launch_par<T_, 16>(KERNEL<T_, 16, M_GEN>, c, __VA_ARGS__);                   \
    }                                                                                              \
  } while (0)

template <typename T, int JB>
static hipError_t step_tiles_t(const sg_ctx* c, const void* act, void* obs, void* rew, uint8_t* done, int tile0,
                               int ntiles, int grid, int add) {
  constexpr size_t lds = use_lds<T, JB>() ? par_lds_bytes<T, JB>() : 0;
  hipError_t e = lds_limit((const void*)k_step_tiles<T, JB>, lds);
  if (e != hipSuccess) return e;
  EnvDev<T> E = env_view<T>(c);
  E.rng_add = (uint32_t)add;
  k_step_tiles<T, JB><<<dim3(grid), kBlk, lds, c->stream>>>(E, c->slot_env, c->tile_dof, tile0, ntiles, (const T*)act,
                                                           (T*)obs, (T*)rew, done);
  return hipGetLastError();
}

template <typename T>
static hipError_t tiles_t(const sg_ctx* c, const void* act, void* obs, void* rew, uint8_t* done, int tile0, int ntiles,
                          int grid, int add) {
  switch (dof_bucket(c->J)) {
    case 1: return step_tiles_t<T, 1>(c, act, obs, rew, done, tile0, ntiles, grid, add);
    case 2: return step_tiles_t<T, 2>(c, act, obs, rew, done, tile0, ntiles, grid, add);
    case 4: return step_tiles_t<T, 4>(c, act, obs, rew, done, tile0, ntiles, grid, add);
    case 7: return step_tiles_t<T, 7>(c, act, obs, rew, done, tile0, ntiles, grid, add);
    case 9: return step_tiles_t<T, 9>(c, act, obs, rew, done, tile0, ntiles, grid, add);
    default: return step_tiles_t<T, 16>(c, act, obs, rew, done, tile0, ntiles, grid, add);
  }
}

template <int J, int M>
static hipError_t step_team_j(const sg_ctx* c, const EnvDev<float>& E, const float* act, float* obs, float* rew,
                              uint8_t* done) {
  constexpr size_t lds = team_step_lds_bytes<J>();
  hipError_t e = lds_limit((const void*)k_step_team<J, M>, lds);
  if (e != hipSuccess) return e;
  k_step_team<J, M><<<dim3((c->N + kBlk - 1) / kBlk), kBlk * kTeam, lds, c->stream>>>(E, act, obs, rew, done);
  return hipGetLastError();
}

// The padded step with a wave team where the context asks for one and the
// chains' bucket has a team kernel (4 to 9 joints); false leaves the
// one-wave kernels.
bool step_team_available(const sg_ctx* c) {
  const int b = dof_bucket(c->J);
  return c->dtype == SG_F32 && b >= 4 && b <= 9;
}

// Auto (team 0): the team while every block is resident at once (two team
// blocks fit a compute unit's LDS; one-wave blocks fit four, so beyond that
// the one-wave kernel needs fewer rounds of blocks).
static bool step_team(const sg_ctx* c, const EnvDev<float>& E, const float* act, float* obs, float* rew,
                      uint8_t* done, hipError_t* err) {
  const int blocks = (c->N + kBlk - 1) / kBlk;
  const bool want = c->team == kTeam || (c->team == 0 && blocks <= 2 * c->n_cu);
  if (!want || c->schedule != SG_SCHED_PADDED || !step_team_available(c)) return false;
  const int b = dof_bucket(c->J);
  if (c->prismatic) {
    *err = b == 4 ? step_team_j<4, M_PRI>(c, E, act, obs, rew, done)
                  : (b == 7 ? step_team_j<7, M_PRI>(c, E, act, obs, rew, done)
                            : step_team_j<9, M_PRI>(c, E, act, obs, rew, done));
  } else if (c->uniform) {
    *err = b == 4 ? step_team_j<4, M_UNI>(c, E, act, obs, rew, done)
                  : (b == 7 ? step_team_j<7, M_UNI>(c, E, act, obs, rew, done)
                            : step_team_j<9, M_UNI>(c, E, act, obs, rew, done));
  } else {
    *err = b == 4 ? step_team_j<4, M_GEN>(c, E, act, obs, rew, done)
                  : (b == 7 ? step_team_j<7, M_GEN>(c, E, act, obs, rew, done)
                            : step_team_j<9, M_GEN>(c, E, act, obs, rew, done));
  }
  return true;
}

// One control step under the context's schedule; the launch that runs last
// advances the noise counter by add.
template <typename T>
static hipError_t step_t(const sg_ctx* c, const void* act, void* obs, void* rew, uint8_t* done, int add) {
  // tiled schedules: FP32 revolute contexts only (sg_set_schedule enforces it)
  if constexpr (sizeof(T) == sizeof(float)) {
    if (c->schedule == SG_SCHED_SORTED) return tiles_t<T>(c, act, obs, rew, done, 0, c->n_tiles, c->n_tiles, add);
    if (c->schedule == SG_SCHED_PERSISTENT) {
      const int grid = c->n_tiles < 512 ? c->n_tiles : 512;
      return tiles_t<T>(c, act, obs, rew, done, 0, c->n_tiles, grid, add);
    }
    if (c->schedule == SG_SCHED_PER_CLASS) {
      for (size_t k = 0; k < c->cls_dof.size(); ++k) {
        const int a = k + 1 == c->cls_dof.size() ? add : 0;
        hipError_t e = tiles_t<T>(c, act, obs, rew, done, c->cls_tile0[k], c->cls_ntiles[k], c->cls_ntiles[k], a);
        if (e != hipSuccess) return e;
      }
      return hipSuccess;
    }
  }
  EnvDev<T> E = env_view<T>(c);
  E.rng_add = (uint32_t)add;
  if constexpr (sizeof(T) == sizeof(float)) {
    hipError_t e = hipSuccess;
    if (step_team(c, E, (const float*)act, (float*)obs, (float*)rew, done, &e)) return e;
  }
  SG_DISPATCH(k_step, T, E, (const T*)act, (T*)obs, (T*)rew, done);
}

template <typename T> static hipError_t observe_t(const sg_ctx* c, void* obs) {
  EnvDev<T> E = env_view<T>(c);
  SG_DISPATCH(k_observe, T, E, (T*)obs);
}
template <typename T>
static hipError_t fd_t(const sg_ctx* c, const void* q, const void* qd, const void* tau, int arm_mode, void* qdd) {
  EnvDev<T> E = env_view<T>(c);
  SG_DISPATCH(k_fd, T, E, (const T*)q, (const T*)qd, (const T*)tau, arm_mode, (T*)qdd);
}
template <typename T>
static hipError_t id_t(const sg_ctx* c, const void* q, const void* qd, const void* qdd, void* tau) {
  EnvDev<T> E = env_view<T>(c);
  SG_DISPATCH(k_id, T, E, (const T*)q, (const T*)qd, (const T*)qdd, (T*)tau);
}
template <typename T> static hipError_t tip_t(const sg_ctx* c, const void* q, void* tip) {
  EnvDev<T> E = env_view<T>(c);
  SG_DISPATCH(k_tip, T, E, (const T*)q, (T*)tip);
}

hipError_t launch_step(const sg_ctx* c, const void* act, void* obs, void* rew, uint8_t* done, int rng_add) {
  return c->dtype == SG_F64 ? step_t<double>(c, act, obs, rew, done, rng_add)
                            : step_t<float>(c, act, obs, rew, done, rng_add);
}
hipError_t launch_observe(const sg_ctx* c, void* obs) {
  return c->dtype == SG_F64 ? observe_t<double>(c, obs) : observe_t<float>(c, obs);
}
hipError_t launch_fd(const sg_ctx* c, const void* q, const void* qd, const void* tau, int arm_mode, void* qdd) {
  return c->dtype == SG_F64 ? fd_t<double>(c, q, qd, tau, arm_mode, qdd) : fd_t<float>(c, q, qd, tau, arm_mode, qdd);
}
hipError_t launch_id(const sg_ctx* c, const void* q, const void* qd, const void* qdd, void* tau) {
  return c->dtype == SG_F64 ? id_t<double>(c, q, qd, qdd, tau) : id_t<float>(c, q, qd, qdd, tau);
}
hipError_t launch_tip(const sg_ctx* c, const void* q, void* tip) {
  return c->dtype == SG_F64 ? tip_t<double>(c, q, tip) : tip_t<float>(c, q, tip);
}
hipError_t launch_reset(const sg_ctx* c) {
  const dim3 g((c->N + 255) / 256);
  if (c->dtype == SG_F64) k_reset<double><<<g, 256, 0, c->stream>>>(env_view<double>(c));
  else k_reset<float><<<g, 256, 0, c->stream>>>(env_view<float>(c));
  if (c->gs) {
    const size_t b = (size_t)c->gs_width * c->N * (c->dtype == SG_F64 ? sizeof(double) : sizeof(float));
    hipError_t e = hipMemcpyAsync(c->gs, c->gs0, b, hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

}  // namespace sgk
