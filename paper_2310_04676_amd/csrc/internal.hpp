// Library-internal context and launcher declarations.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/surgym.h"
#include "env.hpp"

struct sg_ctx {
  int device = 0;
  int n_cu = 256;  // compute units of the device
  int N = 0, J = 0, dtype = SG_F32, S = 1;
  bool uniform = false;    // every env has J joints and J is a kernel instantiation
  bool prismatic = false;  // some env has a prismatic joint
  int task = 0, K = 0, dwell = 1, ep_len = 0;
  int chains = 1;  // chains per env (consecutive env indices)
  double dt = 0, g[3] = {0, 0, 0};
  uint64_t seed = 0;
  // noise counter (control steps drawn so far) and the completion count the
  // kernel advancing it uses: device memory, so captured calls advance it
  uint64_t* rng_dev = nullptr;
  unsigned* rng_tick = nullptr;
  hipStream_t stream = nullptr;
  // device memory (dtype-typed unless noted)
  void* par = nullptr;      // [P_NFIELDS][J][N]
  void* tip = nullptr;      // [3][N]
  void* tip0 = nullptr;     // [3][N] tool tip at q0
  int* nd = nullptr;        // [N]
  void* target = nullptr;   // [3][N]
  void* wp = nullptr;       // [K][3][N]
  int* prog0 = nullptr;     // [N]
  void* q = nullptr;        // [J][N]
  void* qd = nullptr;       // [J][N]
  int* prog = nullptr;      // [N]
  // tracking task: goal state [9][N] (goal, goal velocity, centre) and its
  // value at create (restored by sg_reset)
  void* gs = nullptr;
  void* gs0 = nullptr;
  int gs_width = 0;  // rows of gs: 9 tracking, 3 re-randomised reach, 1 re-randomised path, 0 none
  // per-episode re-randomisation of the reach target / path waypoint set
  int rerand = 0, n_banks = 1;
  double rand_c[3] = {0, 0, 0}, rand_half = 0;
  double trk_sigma = 0, trk_offset = 0, trk_reset_std = 0, trk_c[3] = {0, 0, 0};
  // DOF-class tiling for uneven batches: slots sorted by n_dof, each class
  // padded to whole 64-slot tiles (slot_env = -1 for padding).
  int schedule = 0;               // SG_SCHED_*
  int team = 0;                   // waves per 64-env block sharing the solve: 1, sgk::kTeam, or 0 (auto)
  std::string tune_key;           // the autotuner's key for this context (device, N, chains, DOF mix, task)
  int n_tiles = 0;
  int* slot_env = nullptr;        // [n_tiles * 64]
  int* tile_dof = nullptr;        // [n_tiles]
  std::vector<int> cls_dof, cls_tile0, cls_ntiles;  // per DOF class (host)
  // policy (FP32 contexts)
  int has_policy = 0, h1 = 0, h2 = 0, h3 = 0, pact = 0;  // policy widths (h3 = 0: two hidden layers), activation
  uint16_t* w_bf16 = nullptr;  // W1 | W2 | W3 row-major BF16
  float* bias = nullptr;       // b1 | b2 | b3
  float* log_std = nullptr;    // [J]
  // adjoint workspace (grown on demand)
  float* adj_ws = nullptr;
  size_t adj_ws_floats = 0;
  std::string err;
};

// Third hidden width of a supported policy architecture (0: two hidden
// layers), or -1 for one the kernels are not built for.
int policy_h3(const sg_policy_arch* a);

namespace sgk {

template <typename T> inline EnvDev<T> env_view(const sg_ctx* c) {
  EnvDev<T> E;
  E.N = c->N; E.J = c->J; E.S = c->S; E.task = c->task; E.K = c->K; E.dwell = c->dwell; E.ep_len = c->ep_len;
  E.chains = c->chains;
  E.dt = (T)c->dt;
  E.h = E.dt / (T)c->S;
  E.g[0] = (T)c->g[0]; E.g[1] = (T)c->g[1]; E.g[2] = (T)c->g[2];
  E.par = (const T*)c->par; E.tip = (const T*)c->tip; E.tip0 = (const T*)c->tip0; E.nd = c->nd;
  E.target = (const T*)c->target; E.wp = (const T*)c->wp; E.prog0 = c->prog0;
  E.q = (T*)c->q; E.qd = (T*)c->qd; E.prog = c->prog;
  E.gs = (T*)c->gs;
  E.trk_sigma = (T)c->trk_sigma; E.trk_offset = (T)c->trk_offset; E.trk_reset_std = (T)c->trk_reset_std;
  for (int k = 0; k < 3; ++k) E.trk_c[k] = (T)c->trk_c[k];
  E.rerand = c->rerand; E.nbank = c->n_banks; E.rhalf = (T)c->rand_half;
  for (int k = 0; k < 3; ++k) E.rc[k] = (T)c->rand_c[k];
  E.seed = c->seed;
  E.rng = c->rng_dev;
  E.tick = c->rng_tick;
  E.rng_add = 0;
  return E;
}

// Kernel instantiations cover these max-DOF values; a context uses the
// smallest one >= its J.
int dof_bucket(int J);

// Raise the dynamic-LDS limit of kernel fn to bytes (when above the 64 KB
// default) on the current device, once per (device, kernel address).
hipError_t lds_limit(const void* fn, size_t bytes);

// Whether the padded step has a wave-team kernel for this context.
bool step_team_available(const sg_ctx* c);

// rng_add: how far the launch advances the device noise counter (sg_step: 1;
// the autotuner's trial steps: 0).
hipError_t launch_step(const sg_ctx* c, const void* act, void* obs, void* rew, uint8_t* done, int rng_add);
hipError_t launch_set_counter(const sg_ctx* c, uint64_t value);
hipError_t launch_observe(const sg_ctx* c, void* obs);
hipError_t launch_fd(const sg_ctx* c, const void* q, const void* qd, const void* tau, int arm_mode, void* qdd);
hipError_t launch_id(const sg_ctx* c, const void* q, const void* qd, const void* qdd, void* tau);
hipError_t launch_tip(const sg_ctx* c, const void* q, void* tip);
hipError_t launch_reset(const sg_ctx* c);

// Learning side (FP32 contexts).
hipError_t launch_adjoint(const sg_ctx* c, int T, int K, const float* act, float* loss, float* g_act, float* g_mass,
                          float* ws);
size_t adjoint_ws_floats(const sg_ctx* c, int T, int K);
hipError_t launch_set_masses(sg_ctx* c, const void* m);

hipError_t launch_policy_forward(const sg_ctx* c, const float* x, int n, float* out);
hipError_t launch_rollout(sg_ctx* c, int T, const sg_rollout_bufs* b);
hipError_t launch_gae(hipStream_t s, int T, int n, const float* rew, const float* val, const uint8_t* done,
                      float gamma, float lam, float* adv, float* ret);

}  // namespace sgk
