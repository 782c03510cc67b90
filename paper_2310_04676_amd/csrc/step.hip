// Environment-step kernels: one environment per lane, state and chain in
// VGPRs, structure-of-arrays global layout so each per-joint field is one
// coalesced 64-lane access.
#include "internal.hpp"

namespace sgk {

constexpr int kBlock = 256;

int dof_bucket(int J) {
  if (J <= 1) return 1;
  if (J <= 2) return 2;
  if (J <= 4) return 4;
  if (J <= 7) return 7;
  if (J <= 9) return 9;
  return 16;
}

template <typename T, int J>
__global__ void __launch_bounds__(kBlock) k_step(EnvDev<T> E, const T* __restrict__ act, T* __restrict__ obs,
                                                 T* __restrict__ rew, uint8_t* __restrict__ done) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= E.N) return;
  const int n = E.nd[e];
  Jp<T> P[J];
  T q[J], qd[J], a[J];
  load_chain<T, J>(E, e, n, P);
  load_state<T, J>(E, e, n, q, qd);
#pragma unroll
  for (int j = 0; j < J; ++j) a[j] = j < n ? act[(size_t)j * E.N + e] : T(0);
  physics<T, J>(E, P, n, a, q, qd);
  int prog = E.prog[e];
  T r;
  const uint8_t d = post_step<T, J>(E, e, n, P, q, qd, prog, &r, obs);
  store_state<T, J>(E, e, n, q, qd, prog);
  rew[e] = r;
  done[e] = d;
}

template <typename T, int J>
__global__ void __launch_bounds__(kBlock) k_observe(EnvDev<T> E, T* __restrict__ obs) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= E.N) return;
  const int n = E.nd[e];
  Jp<T> P[J];
  T q[J], qd[J];
  load_chain<T, J>(E, e, n, P);
  load_state<T, J>(E, e, n, q, qd);
  const T tipl[3] = {E.tip[e], E.tip[E.N + e], E.tip[2 * E.N + e]};
  T tip[3], g[3];
  tip_fk<T, J>(P, n, q, tipl, tip);
  goal_of(E, e, E.prog[e], g);
  write_obs<T, J>(E, e, n, q, qd, tip, g, obs);
}

template <typename T, int J>
__global__ void __launch_bounds__(kBlock) k_fd(EnvDev<T> E, const T* __restrict__ qin, const T* __restrict__ qdin,
                                               const T* __restrict__ tauin, int arm_mode, T* __restrict__ qddout) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= E.N) return;
  const int n = E.nd[e];
  Jp<T> P[J];
  T q[J], qd[J], tau[J], arm[J], qdd[J];
  load_chain<T, J>(E, e, n, P);
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const size_t i = (size_t)j * E.N + e;
    q[j] = j < n ? qin[i] : T(0);
    qd[j] = j < n ? qdin[i] : T(0);
    tau[j] = j < n ? tauin[i] : T(0);
    arm[j] = (j < n && arm_mode == SG_ARM_DRIVE) ? E.h * P[j].kd + E.h * E.h * P[j].kp : T(0);
  }
  aba<T, J>(P, n, q, qd, tau, arm, E.g, qdd);
#pragma unroll
  for (int j = 0; j < J; ++j)
    if (j < E.J) qddout[(size_t)j * E.N + e] = j < n ? qdd[j] : T(0);
}

template <typename T, int J>
__global__ void __launch_bounds__(kBlock) k_id(EnvDev<T> E, const T* __restrict__ qin, const T* __restrict__ qdin,
                                               const T* __restrict__ qddin, T* __restrict__ tauout) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= E.N) return;
  const int n = E.nd[e];
  Jp<T> P[J];
  T q[J], qd[J], qdd[J], tau[J];
  load_chain<T, J>(E, e, n, P);
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const size_t i = (size_t)j * E.N + e;
    q[j] = j < n ? qin[i] : T(0);
    qd[j] = j < n ? qdin[i] : T(0);
    qdd[j] = j < n ? qddin[i] : T(0);
  }
  rnea<T, J>(P, n, q, qd, qdd, E.g, tau);
#pragma unroll
  for (int j = 0; j < J; ++j)
    if (j < E.J) tauout[(size_t)j * E.N + e] = j < n ? tau[j] : T(0);
}

template <typename T, int J>
__global__ void __launch_bounds__(kBlock) k_tip(EnvDev<T> E, const T* __restrict__ qin, T* __restrict__ out) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= E.N) return;
  const int n = E.nd[e];
  Jp<T> P[J];
  T q[J];
  load_chain<T, J>(E, e, n, P);
#pragma unroll
  for (int j = 0; j < J; ++j) q[j] = j < n ? qin[(size_t)j * E.N + e] : T(0);
  const T tipl[3] = {E.tip[e], E.tip[E.N + e], E.tip[2 * E.N + e]};
  T tip[3];
  tip_fk<T, J>(P, n, q, tipl, tip);
  out[e] = tip[0];
  out[E.N + e] = tip[1];
  out[2 * E.N + e] = tip[2];
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_reset(EnvDev<T> E) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= E.N) return;
  for (int j = 0; j < E.J; ++j) {
    const size_t i = (size_t)j * E.N + e;
    E.q[i] = E.par[(size_t)P_Q0 * E.J * E.N + i];
    E.qd[i] = T(0);
  }
  E.prog[e] = E.prog0[e];
}

static inline dim3 grid_for(int N) { return dim3((N + kBlock - 1) / kBlock); }

#define SG_DISPATCH_J(J_, CALL)          \
  switch (dof_bucket(J_)) {              \
    case 1: { constexpr int JJ = 1; CALL; break; } \
    case 2: { constexpr int JJ = 2; CALL; break; } \
    case 4: { constexpr int JJ = 4; CALL; break; } \
    case 7: { constexpr int JJ = 7; CALL; break; } \
    case 9: { constexpr int JJ = 9; CALL; break; } \
    default: { constexpr int JJ = 16; CALL; break; } \
  }

template <typename T>
static hipError_t step_t(const sg_ctx* c, const void* act, void* obs, void* rew, uint8_t* done) {
  EnvDev<T> E = env_view<T>(c);
  SG_DISPATCH_J(c->J, (k_step<T, JJ><<<grid_for(c->N), kBlock, 0, c->stream>>>(E, (const T*)act, (T*)obs, (T*)rew, done)));
  return hipGetLastError();
}

template <typename T> static hipError_t observe_t(const sg_ctx* c, void* obs) {
  EnvDev<T> E = env_view<T>(c);
  SG_DISPATCH_J(c->J, (k_observe<T, JJ><<<grid_for(c->N), kBlock, 0, c->stream>>>(E, (T*)obs)));
  return hipGetLastError();
}

template <typename T>
static hipError_t fd_t(const sg_ctx* c, const void* q, const void* qd, const void* tau, int arm_mode, void* qdd) {
  EnvDev<T> E = env_view<T>(c);
  SG_DISPATCH_J(c->J, (k_fd<T, JJ><<<grid_for(c->N), kBlock, 0, c->stream>>>(E, (const T*)q, (const T*)qd, (const T*)tau, arm_mode, (T*)qdd)));
  return hipGetLastError();
}

template <typename T>
static hipError_t id_t(const sg_ctx* c, const void* q, const void* qd, const void* qdd, void* tau) {
  EnvDev<T> E = env_view<T>(c);
  SG_DISPATCH_J(c->J, (k_id<T, JJ><<<grid_for(c->N), kBlock, 0, c->stream>>>(E, (const T*)q, (const T*)qd, (const T*)qdd, (T*)tau)));
  return hipGetLastError();
}

template <typename T> static hipError_t tip_t(const sg_ctx* c, const void* q, void* tip) {
  EnvDev<T> E = env_view<T>(c);
  SG_DISPATCH_J(c->J, (k_tip<T, JJ><<<grid_for(c->N), kBlock, 0, c->stream>>>(E, (const T*)q, (T*)tip)));
  return hipGetLastError();
}

hipError_t launch_step(const sg_ctx* c, const void* act, void* obs, void* rew, uint8_t* done) {
  return c->dtype == SG_F64 ? step_t<double>(c, act, obs, rew, done) : step_t<float>(c, act, obs, rew, done);
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
  if (c->dtype == SG_F64) k_reset<double><<<grid_for(c->N), kBlock, 0, c->stream>>>(env_view<double>(c));
  else k_reset<float><<<grid_for(c->N), kBlock, 0, c->stream>>>(env_view<float>(c));
  return hipGetLastError();
}

}  // namespace sgk
