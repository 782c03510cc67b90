// C interface: argument checking, context setup (host-side conversion of the
// robot description to the device parameter block), and dispatch.
#include <stdio.h>
#include <string.h>

#include <cmath>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <utility>
#include <vector>

#include "internal.hpp"
#include "mlp.hpp"

namespace {

thread_local std::string g_create_err;

sg_status fail(sg_ctx* c, sg_status s, const std::string& msg) {
  if (c) c->err = msg;
  else g_create_err = msg;
  return s;
}

sg_status hip_fail(sg_ctx* c, hipError_t e, const char* where) {
  return fail(c, SG_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

bool aligned(const void* p) { return ((uintptr_t)p & 15u) == 0; }

template <typename T> hipError_t upload(void** dst, const std::vector<double>& src) {
  std::vector<T> tmp(src.size());
  for (size_t i = 0; i < src.size(); ++i) tmp[i] = (T)src[i];
  hipError_t e = hipMalloc(dst, tmp.size() * sizeof(T) + 16);
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice);
}

void free_ctx(sg_ctx* c) {
  void* ptrs[] = {c->par, c->tip, c->tip0, c->nd, c->target, c->wp, c->prog0, c->q, c->qd, c->prog, c->w_bf16, c->bias,
                  c->log_std, c->slot_env, c->tile_dof, c->adj_ws, c->gs, c->gs0, c->rng_dev};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
}

}  // namespace

namespace {

// Autotuner choices remembered for the rest of the process, keyed by what the
// step's cost depends on: the device's architecture, N, the number type, the
// chain shape (max joints, prismatic joints, chains per env), the task and
// the histogram of joint counts. Value: (schedule, waves per block).
std::mutex g_tune_mu;
std::map<std::string, std::pair<int, int>> g_tune;

std::string tuning_key(const sg_ctx* c, const int32_t* n_dof) {
  hipDeviceProp_t prop;
  std::string arch = "gpu";
  if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) {
    arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);
  }
  std::vector<int> hist(c->J + 1, 0);
  for (int e = 0; e < c->N; ++e) hist[n_dof[e]] += 1;
  std::ostringstream k;
  k << arch << "|n=" << c->N << "|" << (c->dtype == SG_F64 ? "f64" : "f32") << "|j=" << c->J
    << "|pr=" << (c->prismatic ? 1 : 0) << "|c=" << c->chains << "|task=" << c->task << "|dof=";
  bool first = true;
  for (int d = 1; d <= c->J; ++d)
    if (hist[d]) {
      k << (first ? "" : ",") << d << "x" << hist[d];
      first = false;
    }
  return k.str();
}

bool schedule_allowed(const sg_ctx* c, int s) {
  if (s < SG_SCHED_PADDED || s > SG_SCHED_PERSISTENT) return false;
  return s == SG_SCHED_PADDED || (c->dtype == SG_F32 && !c->prismatic && c->chains == 1);
}

bool team_allowed(const sg_ctx* c, int w) { return w == 1 || (w == sgk::kTeam && c->dtype == SG_F32); }

// The policy's weight and bias images (the layout of mlp.hpp, through
// img_source) from per-layer BF16 weights and FP32 biases.
template <int H3>
void pack_policy_host(int W, int O, const uint16_t* const* Wl, const float* const* bl, std::vector<uint16_t>& img,
                      std::vector<float>& bimg) {
  using S = sgk::PolicyShape<H3>;
  const int in[4] = {W, sgk::kH1, sgk::kH2, H3 ? H3 : sgk::kH2};
  const int lo = H3 ? 3 : 2;  // index of the output layer among Wl
  img.assign((size_t)S::kWFrags * 8, 0);
  for (int f = 0; f < S::kWFrags / 64; ++f)
    for (int l = 0; l < 64; ++l)
      for (int s = 0; s < 8; ++s) {
        int layer, row, k;
        if (!sgk::img_source<H3>(f, l, s, W, O, &layer, &row, &k)) continue;
        const int L = layer == 3 ? lo : layer;
        const int K = layer == 3 ? in[3] : in[layer];
        img[((size_t)f * 64 + l) * 8 + s] = Wl[L][(size_t)row * K + k];
      }
  bimg.assign(S::kBias, 0.f);
  for (int i = 0; i < sgk::kH1; ++i) bimg[i] = bl[0][i];
  for (int i = 0; i < sgk::kH2; ++i) bimg[sgk::kH1 + i] = bl[1][i];
  for (int i = 0; i < H3; ++i) bimg[sgk::kH1 + sgk::kH2 + i] = bl[2][i];
  for (int i = 0; i < O; ++i) bimg[sgk::kH1 + sgk::kH2 + H3 + i] = bl[lo][i];
}

}  // namespace

// The two networks the kernels are built for; 0 for the 256-128 tanh one,
// 64 (its third width) for the 256-128-64 ELU one, -1 otherwise.
int policy_h3(const sg_policy_arch* a) {
  if (!a) return -1;
  if (a->n_hidden == 2 && a->hidden[0] == 256 && a->hidden[1] == 128 && a->act == SG_ACT_TANH) return 0;
  if (a->n_hidden == 3 && a->hidden[0] == 256 && a->hidden[1] == 128 && a->hidden[2] == 64 && a->act == SG_ACT_ELU)
    return 64;
  return -1;
}

extern "C" {

const char* sg_version(void) { return "surgym-mi355x 0.1 (gfx950)"; }

const char* sg_last_error(const sg_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_err.c_str(); }

sg_status sg_create(const sg_robot_desc* r, const sg_task_desc* t, sg_ctx** out) {
  g_create_err.clear();
  if (!r || !t || !out) return fail(nullptr, SG_E_INVAL, "sg_create: null argument");
  *out = nullptr;
  const int N = r->n_env, J = r->max_dof;
  if (N < 1) return fail(nullptr, SG_E_INVAL, "sg_create: n_env must be >= 1");
  if (J < 1 || J > SG_MAX_DOF) return fail(nullptr, SG_E_UNSUPPORTED, "sg_create: max_dof must be in 1..16");
  if (r->dtype != SG_F32 && r->dtype != SG_F64) return fail(nullptr, SG_E_INVAL, "sg_create: bad dtype");
  if (!r->n_dof || !r->axis || !r->offset || !r->com || !r->mass || !r->inertia || !r->kp || !r->kd || !r->q_lo ||
      !r->q_hi || !r->q0 || !r->tip)
    return fail(nullptr, SG_E_INVAL, "sg_create: null robot array");
  if (!(r->dt > 0) || r->substeps < 1) return fail(nullptr, SG_E_INVAL, "sg_create: dt must be > 0, substeps >= 1");
  if (t->task != SG_TASK_REACH && t->task != SG_TASK_PATH && t->task != SG_TASK_TRACK)
    return fail(nullptr, SG_E_INVAL, "sg_create: bad task");
  if ((t->task == SG_TASK_REACH || t->task == SG_TASK_TRACK) && !t->target)
    return fail(nullptr, SG_E_INVAL, "sg_create: reach and tracking tasks need target");
  if (t->task == SG_TASK_TRACK && (!(t->track_sigma >= 0) || !(t->track_offset > 0) || !(t->track_reset_std >= 0)))
    return fail(nullptr, SG_E_INVAL, "sg_create: tracking needs sigma >= 0, offset > 0, reset_std >= 0");
  if (t->task == SG_TASK_PATH &&
      (!t->waypoints || t->n_waypoints < 1 || t->n_waypoints > SG_MAX_WAYPOINTS || t->dwell < 1))
    return fail(nullptr, SG_E_INVAL, "sg_create: path task needs 1..32 waypoints and dwell >= 1");
  const int n_banks = t->n_banks > 1 ? t->n_banks : 1;
  if (t->rerandomize) {
    if (t->task == SG_TASK_TRACK)
      return fail(nullptr, SG_E_INVAL, "sg_create: tracking re-draws its goals already (rerandomize is for reach/path)");
    if (t->chains_per_env > 1)
      return fail(nullptr, SG_E_UNSUPPORTED, "sg_create: rerandomize needs one chain per env");
    if (t->task == SG_TASK_REACH && !(t->rand_half_width > 0))
      return fail(nullptr, SG_E_INVAL, "sg_create: rerandomize (reach) needs rand_half_width > 0");
    if (t->task == SG_TASK_PATH && n_banks > 64) return fail(nullptr, SG_E_INVAL, "sg_create: n_banks must be 1..64");
  } else if (n_banks != 1) {
    return fail(nullptr, SG_E_INVAL, "sg_create: several waypoint sets need rerandomize");
  }
  const int C = t->chains_per_env > 1 ? t->chains_per_env : 1;
  if (C != 1 && C != 2 && C != 4) return fail(nullptr, SG_E_UNSUPPORTED, "sg_create: chains_per_env must be 1, 2 or 4");
  if (N % C) return fail(nullptr, SG_E_INVAL, "sg_create: n_env must be a multiple of chains_per_env");
  if (C > 1 && t->progress0)
    for (int e = 0; e < N; ++e)
      if (t->progress0[e] != t->progress0[e - e % C])
        return fail(nullptr, SG_E_INVAL, "sg_create: the chains of an env must share progress0");
  const size_t JN = (size_t)J * N;
  for (int e = 0; e < N; ++e) {
    const int n = r->n_dof[e];
    if (n < 1 || n > J) return fail(nullptr, SG_E_INVAL, "sg_create: n_dof out of 1..max_dof");
    for (int j = 0; j < n; ++j) {
      const size_t i = (size_t)j * N + e;
      const double ax = r->axis[i], ay = r->axis[JN + i], az = r->axis[2 * JN + i];
      if (std::fabs(ax * ax + ay * ay + az * az - 1.0) > 1e-6)
        return fail(nullptr, SG_E_INVAL, "sg_create: joint axis not unit length");
      if (!(r->mass[i] > 0)) return fail(nullptr, SG_E_INVAL, "sg_create: link mass must be > 0");
      if (!(r->q_hi[i] > r->q_lo[i])) return fail(nullptr, SG_E_INVAL, "sg_create: q_hi must exceed q_lo");
      if (r->kp[i] < 0 || r->kd[i] < 0) return fail(nullptr, SG_E_INVAL, "sg_create: gains must be >= 0");
      if (r->joint_type && r->joint_type[i] != SG_JOINT_REVOLUTE && r->joint_type[i] != SG_JOINT_PRISMATIC)
        return fail(nullptr, SG_E_INVAL, "sg_create: joint_type must be 0 (revolute) or 1 (prismatic)");
    }
  }
  sg_ctx* c = new sg_ctx();
  hipError_t he = hipGetDevice(&c->device);
  if (he == hipSuccess) he = hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, c->device);
  if (he != hipSuccess) {
    delete c;
    return hip_fail(nullptr, he, "hipGetDevice");
  }
  c->N = N; c->J = J; c->dtype = r->dtype; c->S = r->substeps; c->dt = r->dt;
  c->uniform = sgk::dof_bucket(J) == J;
  for (int e = 0; e < N && c->uniform; ++e) c->uniform = r->n_dof[e] == J;
  for (int k = 0; k < 3; ++k) c->g[k] = r->gravity[k];
  c->task = t->task; c->K = t->task == SG_TASK_PATH ? t->n_waypoints : 1;
  c->dwell = t->dwell > 0 ? t->dwell : 1; c->ep_len = t->ep_len; c->seed = t->seed;
  c->chains = C;
  if (t->task == SG_TASK_TRACK) {
    c->trk_sigma = t->track_sigma; c->trk_offset = t->track_offset; c->trk_reset_std = t->track_reset_std;
    for (int k = 0; k < 3; ++k) c->trk_c[k] = t->track_centre[k];
  }
  if (t->rerandomize) {
    c->rerand = 1;
    c->n_banks = t->task == SG_TASK_PATH ? n_banks : 1;
    c->rand_half = t->rand_half_width;
    for (int k = 0; k < 3; ++k) c->rand_c[k] = t->rand_centre[k];
  }

  // Device parameter block [P_NFIELDS][J][N]; padded joints stay zero.
  std::vector<double> par((size_t)sgk::P_NFIELDS * JN, 0.0);
  auto P = [&](int f, size_t i) -> double& { return par[(size_t)f * JN + i]; };
  for (int e = 0; e < N; ++e) {
    for (int j = 0; j < r->n_dof[e]; ++j) {
      const size_t i = (size_t)j * N + e;
      const double m = r->mass[i];
      const double cx = r->com[i], cy = r->com[JN + i], cz = r->com[2 * JN + i];
      const double* I = r->inertia;
      const double c2 = cx * cx + cy * cy + cz * cz;
      P(sgk::P_AX, i) = r->axis[i]; P(sgk::P_AY, i) = r->axis[JN + i]; P(sgk::P_AZ, i) = r->axis[2 * JN + i];
      P(sgk::P_OX, i) = r->offset[i]; P(sgk::P_OY, i) = r->offset[JN + i]; P(sgk::P_OZ, i) = r->offset[2 * JN + i];
      P(sgk::P_M, i) = m;
      P(sgk::P_HX, i) = m * cx; P(sgk::P_HY, i) = m * cy; P(sgk::P_HZ, i) = m * cz;
      // rotational inertia about the link origin: I_c + m (|c|^2 1 - c c^T)
      P(sgk::P_IXX, i) = I[i] + m * (c2 - cx * cx);
      P(sgk::P_IYY, i) = I[JN + i] + m * (c2 - cy * cy);
      P(sgk::P_IZZ, i) = I[2 * JN + i] + m * (c2 - cz * cz);
      P(sgk::P_IXY, i) = I[3 * JN + i] - m * cx * cy;
      P(sgk::P_IXZ, i) = I[4 * JN + i] - m * cx * cz;
      P(sgk::P_IYZ, i) = I[5 * JN + i] - m * cy * cz;
      P(sgk::P_KP, i) = r->kp[i]; P(sgk::P_KD, i) = r->kd[i];
      P(sgk::P_LO, i) = r->q_lo[i]; P(sgk::P_HI, i) = r->q_hi[i];
      P(sgk::P_Q0, i) = r->q0[i];
      if (r->joint_type && r->joint_type[i] == SG_JOINT_PRISMATIC) {
        P(sgk::P_PR, i) = 1.0;
        c->prismatic = true;
      }
    }
  }
  std::vector<double> tip(r->tip, r->tip + 3 * (size_t)N);
  std::vector<double> tgt(3 * (size_t)N, 0.0), wps;
  if (t->target) tgt.assign(t->target, t->target + 3 * (size_t)N);
  if (t->task == SG_TASK_PATH) wps.assign(t->waypoints, t->waypoints + (size_t)c->n_banks * c->K * 3 * N);
  else wps.assign(3 * (size_t)N, 0.0);
  std::vector<int> nd(r->n_dof, r->n_dof + N), prog0(N, 0);
  // DOF-class tiles: envs of each class in env order, padded to 64 slots
  std::vector<int> slot_env, tile_dof;
  for (int d = 1; d <= J; ++d) {
    std::vector<int> members;
    for (int e = 0; e < N; ++e)
      if (nd[e] == d) members.push_back(e);
    if (members.empty()) continue;
    const int nt = ((int)members.size() + 63) / 64;
    c->cls_dof.push_back(d);
    c->cls_tile0.push_back((int)tile_dof.size());
    c->cls_ntiles.push_back(nt);
    for (int t = 0; t < nt; ++t) tile_dof.push_back(d);
    members.resize((size_t)nt * 64, -1);
    slot_env.insert(slot_env.end(), members.begin(), members.end());
  }
  c->n_tiles = (int)tile_dof.size();
  if (t->progress0) prog0.assign(t->progress0, t->progress0 + N);

  auto up = [&](void** d, const std::vector<double>& v) {
    return c->dtype == SG_F64 ? upload<double>(d, v) : upload<float>(d, v);
  };
  hipError_t e = hipSuccess;
  const size_t esz = c->dtype == SG_F64 ? sizeof(double) : sizeof(float);
  if (e == hipSuccess) e = up(&c->par, par);
  if (e == hipSuccess) e = up(&c->tip, tip);
  if (e == hipSuccess) e = up(&c->target, tgt);
  if (e == hipSuccess) e = up(&c->wp, wps);
  if (e == hipSuccess && t->task == SG_TASK_TRACK) {
    // goal on the first episode's centre (the target), at rest
    std::vector<double> gs0(9 * (size_t)N, 0.0);
    for (int k = 0; k < 3; ++k)
      for (int i = 0; i < N; ++i) gs0[k * (size_t)N + i] = gs0[(6 + k) * (size_t)N + i] = tgt[k * (size_t)N + i];
    e = up(&c->gs0, gs0);
    if (e == hipSuccess) e = up(&c->gs, gs0);
    c->gs_width = 9;
  } else if (e == hipSuccess && c->rerand) {
    // reach: the first episode's target; path: waypoint set 0
    c->gs_width = t->task == SG_TASK_REACH ? 3 : 1;
    std::vector<double> gs0((size_t)c->gs_width * N, 0.0);
    if (t->task == SG_TASK_REACH) gs0 = tgt;
    e = up(&c->gs0, gs0);
    if (e == hipSuccess) e = up(&c->gs, gs0);
  }
  if (e == hipSuccess) e = hipMalloc((void**)&c->nd, N * sizeof(int));
  if (e == hipSuccess) e = hipMemcpy(c->nd, nd.data(), N * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc((void**)&c->prog0, N * sizeof(int));
  if (e == hipSuccess) e = hipMemcpy(c->prog0, prog0.data(), N * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc((void**)&c->prog, N * sizeof(int));
  if (e == hipSuccess) e = hipMalloc((void**)&c->slot_env, slot_env.size() * sizeof(int));
  if (e == hipSuccess)
    e = hipMemcpy(c->slot_env, slot_env.data(), slot_env.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc((void**)&c->tile_dof, tile_dof.size() * sizeof(int));
  if (e == hipSuccess)
    e = hipMemcpy(c->tile_dof, tile_dof.data(), tile_dof.size() * sizeof(int), hipMemcpyHostToDevice);
  // the noise counter (8 bytes) and its completion count (4 bytes), zeroed
  if (e == hipSuccess) e = hipMalloc((void**)&c->rng_dev, 16);
  if (e == hipSuccess) e = hipMemset(c->rng_dev, 0, 16);
  if (e == hipSuccess) c->rng_tick = reinterpret_cast<unsigned*>(c->rng_dev + 1);
  if (e == hipSuccess) e = hipMalloc(&c->q, JN * esz);
  if (e == hipSuccess) e = hipMalloc(&c->qd, JN * esz);
  if (e == hipSuccess) e = hipMemset(c->q, 0, JN * esz);
  if (e == hipSuccess) e = hipMemset(c->qd, 0, JN * esz);
  // the tool tip at q0 (the pose a reset returns to), for the step's resets
  if (e == hipSuccess) e = hipMalloc(&c->tip0, 3 * (size_t)N * esz);
  if (e == hipSuccess)
    e = sgk::launch_tip(c, static_cast<const char*>(c->par) + (size_t)sgk::P_Q0 * J * N * esz, c->tip0);
  if (e == hipSuccess) e = sgk::launch_reset(c);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    free_ctx(c);
    delete c;
    return hip_fail(nullptr, e, "sg_create");
  }
  // a choice the autotuner made for a context of the same key
  c->tune_key = tuning_key(c, r->n_dof);
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    const auto it = g_tune.find(c->tune_key);
    if (it != g_tune.end() && schedule_allowed(c, it->second.first) && team_allowed(c, it->second.second)) {
      c->schedule = it->second.first;
      c->team = it->second.second;
    }
  }
  *out = c;
  return SG_OK;
}

void sg_destroy(sg_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  free_ctx(c);
  delete c;
}

sg_status sg_set_stream(sg_ctx* c, void* s) {
  if (!c) return SG_E_INVAL;
  c->stream = (hipStream_t)s;
  return SG_OK;
}

sg_status sg_synchronize(sg_ctx* c) {
  if (!c) return SG_E_INVAL;
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess) e = hipGetLastError();
  return e == hipSuccess ? SG_OK : hip_fail(c, e, "sg_synchronize");
}

sg_status sg_reset(sg_ctx* c) {
  if (!c) return SG_E_INVAL;
  hipError_t e = sgk::launch_reset(c);
  if (e == hipSuccess) e = sgk::launch_set_counter(c, 0);
  return e == hipSuccess ? SG_OK : hip_fail(c, e, "sg_reset");
}

sg_status sg_step(sg_ctx* c, const void* act, void* obs, void* rew, uint8_t* done) {
  if (!c) return SG_E_INVAL;
  if (!act || !obs || !rew || !done) return fail(c, SG_E_INVAL, "sg_step: null buffer");
  if (!aligned(act) || !aligned(obs) || !aligned(rew)) return fail(c, SG_E_INVAL, "sg_step: misaligned buffer");
  if (act == obs || act == rew) return fail(c, SG_E_INVAL, "sg_step: outputs alias actions");
  hipError_t e = sgk::launch_step(c, act, obs, rew, done, 1);
  return e == hipSuccess ? SG_OK : hip_fail(c, e, "sg_step");
}

sg_status sg_set_schedule(sg_ctx* c, int32_t schedule) {
  if (!c) return SG_E_INVAL;
  if (schedule < SG_SCHED_PADDED || schedule > SG_SCHED_PERSISTENT)
    return fail(c, SG_E_INVAL, "sg_set_schedule: unknown schedule");
  if (schedule != SG_SCHED_PADDED && c->dtype != SG_F32)
    return fail(c, SG_E_UNSUPPORTED, "sg_set_schedule: tiled schedules need an FP32 context");
  if (schedule != SG_SCHED_PADDED && c->prismatic)
    return fail(c, SG_E_UNSUPPORTED, "sg_set_schedule: tiled schedules need an all-revolute context");
  if (schedule != SG_SCHED_PADDED && c->chains > 1)
    return fail(c, SG_E_UNSUPPORTED, "sg_set_schedule: tiled schedules need one chain per env");
  c->schedule = schedule;
  return SG_OK;
}

sg_status sg_get_schedule(const sg_ctx* c, int32_t* schedule) {
  if (!c || !schedule) return SG_E_INVAL;
  *schedule = c->schedule;
  return SG_OK;
}

sg_status sg_set_team(sg_ctx* c, int32_t waves) {
  if (!c) return SG_E_INVAL;
  if (waves != 0 && waves != 1 && waves != sgk::kTeam) return fail(c, SG_E_INVAL, "sg_set_team: waves must be 0, 1 or 4");
  if (waves == sgk::kTeam && c->dtype != SG_F32)
    return fail(c, SG_E_UNSUPPORTED, "sg_set_team: wave teams need an FP32 context");
  c->team = waves;
  return SG_OK;
}

sg_status sg_get_team(const sg_ctx* c, int32_t* waves) {
  if (!c || !waves) return SG_E_INVAL;
  *waves = c->team;
  return SG_OK;
}

sg_status sg_autotune_step(sg_ctx* c, const void* act, int32_t trials, int32_t* best, int32_t* best_team,
                           float* ms_per_step) {
  if (!c) return SG_E_INVAL;
  if (!act || !aligned(act) || trials < 1 || trials > 10000) return fail(c, SG_E_INVAL, "sg_autotune_step: bad argument");
  const size_t esz = c->dtype == SG_F64 ? sizeof(double) : sizeof(float);
  const size_t JN = (size_t)c->J * c->N, W = 2 * (size_t)c->J + 10;
  void *q = nullptr, *qd = nullptr, *obs = nullptr, *rew = nullptr;
  int* pr = nullptr;
  uint8_t* done = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc(&q, JN * esz);
  if (e == hipSuccess) e = hipMalloc(&qd, JN * esz);
  if (e == hipSuccess) e = hipMalloc((void**)&pr, c->N * sizeof(int));
  if (e == hipSuccess) e = hipMalloc(&obs, W * c->N * esz);
  if (e == hipSuccess) e = hipMalloc(&rew, c->N * esz);
  if (e == hipSuccess) e = hipMalloc((void**)&done, c->N);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  // save the state; every candidate starts from it and it is restored after
  if (e == hipSuccess) e = hipMemcpyAsync(q, c->q, JN * esz, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(qd, c->qd, JN * esz, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(pr, c->prog, c->N * sizeof(int), hipMemcpyDeviceToDevice, c->stream);
  void* gsv = nullptr;
  const size_t gsb = (size_t)c->gs_width * c->N * esz;
  if (e == hipSuccess && c->gs) e = hipMalloc(&gsv, gsb);
  if (e == hipSuccess && c->gs) e = hipMemcpyAsync(gsv, c->gs, gsb, hipMemcpyDeviceToDevice, c->stream);
  const int saved = c->schedule, saved_team = c->team;
  // candidates: the four schedules with one wave per 64 envs, then the
  // padded schedule with a wave team
  const int sched[5] = {SG_SCHED_PADDED, SG_SCHED_SORTED, SG_SCHED_PER_CLASS, SG_SCHED_PERSISTENT, SG_SCHED_PADDED};
  const int team[5] = {1, 1, 1, 1, sgk::kTeam};
  float best_ms = 0.f;
  int best_k = 0;
  for (int k = 0; k < 5 && e == hipSuccess; ++k) {
    if (ms_per_step) ms_per_step[k] = -1.f;
    if (!schedule_allowed(c, sched[k]) || !team_allowed(c, team[k])) continue;
    if (team[k] != 1 && !sgk::step_team_available(c)) continue;
    c->schedule = sched[k];
    c->team = team[k];
    for (int i = 0; i <= trials && e == hipSuccess; ++i) {
      if (i == 1) e = hipEventRecord(e0, c->stream);
      if (e == hipSuccess) e = sgk::launch_step(c, act, obs, rew, done, 0);
    }
    if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    ms /= (float)trials;
    if (ms_per_step) ms_per_step[k] = ms;
    if (k == 0 || ms < best_ms) {
      best_ms = ms;
      best_k = k;
    }
    if (e == hipSuccess) e = hipMemcpyAsync(c->q, q, JN * esz, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->qd, qd, JN * esz, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->prog, pr, c->N * sizeof(int), hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess && c->gs) e = hipMemcpyAsync(c->gs, gsv, gsb, hipMemcpyDeviceToDevice, c->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  c->schedule = e == hipSuccess ? sched[best_k] : saved;
  c->team = e == hipSuccess ? team[best_k] : saved_team;
  if (e == hipSuccess) {
    if (best) *best = sched[best_k];
    if (best_team) *best_team = team[best_k];
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune[c->tune_key] = {sched[best_k], team[best_k]};
  }
  if (gsv) (void)hipFree(gsv);
  void* ptrs[] = {q, qd, pr, obs, rew, done};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return e == hipSuccess ? SG_OK : hip_fail(c, e, "sg_autotune_step");
}

sg_status sg_tuning_export(char* buf, size_t cap, size_t* len) {
  if (!len || (cap && !buf)) return SG_E_INVAL;
  std::string text;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    for (const auto& kv : g_tune)
      text += kv.first + " " + std::to_string(kv.second.first) + " " + std::to_string(kv.second.second) + "\n";
  }
  *len = text.size() + 1;
  if (cap) {
    const size_t n = text.size() < cap - 1 ? text.size() : cap - 1;
    memcpy(buf, text.data(), n);
    buf[n] = 0;
  }
  return SG_OK;
}

sg_status sg_tuning_import(const char* text) {
  if (!text) return SG_E_INVAL;
  std::istringstream in(text);
  std::string line;
  while (std::getline(in, line)) {
    if (line.empty()) continue;
    std::istringstream ls(line);
    std::string key, rest;
    int s = -1, w = -1;
    if (!(ls >> key >> s >> w) || (ls >> rest) || s < SG_SCHED_PADDED || s > SG_SCHED_PERSISTENT ||
        (w != 1 && w != sgk::kTeam))
      return fail(nullptr, SG_E_INVAL, "sg_tuning_import: malformed line");
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune[key] = {s, w};
  }
  return SG_OK;
}

sg_status sg_observe(sg_ctx* c, void* obs) {
  if (!c) return SG_E_INVAL;
  if (!obs || !aligned(obs)) return fail(c, SG_E_INVAL, "sg_observe: null or misaligned buffer");
  hipError_t e = sgk::launch_observe(c, obs);
  return e == hipSuccess ? SG_OK : hip_fail(c, e, "sg_observe");
}

sg_status sg_get_state(sg_ctx* c, void* q, void* qd, int32_t* progress, uint64_t* rng_step) {
  if (!c) return SG_E_INVAL;
  const size_t esz = c->dtype == SG_F64 ? sizeof(double) : sizeof(float);
  const size_t JN = (size_t)c->J * c->N;
  hipError_t e = hipSuccess;
  if (q && e == hipSuccess) e = hipMemcpyAsync(q, c->q, JN * esz, hipMemcpyDeviceToDevice, c->stream);
  if (qd && e == hipSuccess) e = hipMemcpyAsync(qd, c->qd, JN * esz, hipMemcpyDeviceToDevice, c->stream);
  if (progress && e == hipSuccess)
    e = hipMemcpyAsync(progress, c->prog, c->N * sizeof(int), hipMemcpyDeviceToDevice, c->stream);
  if (rng_step && e == hipSuccess) {
    uint64_t v = 0;
    e = hipMemcpyAsync(&v, c->rng_dev, sizeof(v), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) *rng_step = v;
  }
  return e == hipSuccess ? SG_OK : hip_fail(c, e, "sg_get_state");
}

sg_status sg_set_state(sg_ctx* c, const void* q, const void* qd, const int32_t* progress, uint64_t rng_step) {
  if (!c) return SG_E_INVAL;
  const size_t esz = c->dtype == SG_F64 ? sizeof(double) : sizeof(float);
  const size_t JN = (size_t)c->J * c->N;
  hipError_t e = hipSuccess;
  if (q && e == hipSuccess) e = hipMemcpyAsync(c->q, q, JN * esz, hipMemcpyDeviceToDevice, c->stream);
  if (qd && e == hipSuccess) e = hipMemcpyAsync(c->qd, qd, JN * esz, hipMemcpyDeviceToDevice, c->stream);
  if (progress && e == hipSuccess)
    e = hipMemcpyAsync(c->prog, progress, c->N * sizeof(int), hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) e = sgk::launch_set_counter(c, rng_step);
  return e == hipSuccess ? SG_OK : hip_fail(c, e, "sg_set_state");
}

sg_status sg_get_goal_state(sg_ctx* c, void* gs) {
  if (!c) return SG_E_INVAL;
  if (!c->gs) return fail(c, SG_E_STATE, "sg_get_goal_state: the task has no goal state");
  if (!gs) return fail(c, SG_E_INVAL, "sg_get_goal_state: null buffer");
  const size_t b = (size_t)c->gs_width * c->N * (c->dtype == SG_F64 ? sizeof(double) : sizeof(float));
  hipError_t e = hipMemcpyAsync(gs, c->gs, b, hipMemcpyDeviceToDevice, c->stream);
  return e == hipSuccess ? SG_OK : hip_fail(c, e, "sg_get_goal_state");
}

sg_status sg_set_goal_state(sg_ctx* c, const void* gs) {
  if (!c) return SG_E_INVAL;
  if (!c->gs) return fail(c, SG_E_STATE, "sg_set_goal_state: the task has no goal state");
  if (!gs) return fail(c, SG_E_INVAL, "sg_set_goal_state: null buffer");
  const size_t b = (size_t)c->gs_width * c->N * (c->dtype == SG_F64 ? sizeof(double) : sizeof(float));
  hipError_t e = hipMemcpyAsync(c->gs, gs, b, hipMemcpyDeviceToDevice, c->stream);
  return e == hipSuccess ? SG_OK : hip_fail(c, e, "sg_set_goal_state");
}

sg_status sg_forward_dynamics(sg_ctx* c, const void* q, const void* qd, const void* tau, int32_t arm_mode, void* qdd) {
  if (!c) return SG_E_INVAL;
  if (!q || !qd || !tau || !qdd) return fail(c, SG_E_INVAL, "sg_forward_dynamics: null buffer");
  if (arm_mode != SG_ARM_NONE && arm_mode != SG_ARM_DRIVE) return fail(c, SG_E_INVAL, "sg_forward_dynamics: bad arm_mode");
  hipError_t e = sgk::launch_fd(c, q, qd, tau, arm_mode, qdd);
  return e == hipSuccess ? SG_OK : hip_fail(c, e, "sg_forward_dynamics");
}

sg_status sg_inverse_dynamics(sg_ctx* c, const void* q, const void* qd, const void* qdd, void* tau) {
  if (!c) return SG_E_INVAL;
  if (!q || !qd || !qdd || !tau) return fail(c, SG_E_INVAL, "sg_inverse_dynamics: null buffer");
  hipError_t e = sgk::launch_id(c, q, qd, qdd, tau);
  return e == hipSuccess ? SG_OK : hip_fail(c, e, "sg_inverse_dynamics");
}

sg_status sg_tip_position(sg_ctx* c, const void* q, void* tip) {
  if (!c) return SG_E_INVAL;
  if (!q || !tip) return fail(c, SG_E_INVAL, "sg_tip_position: null buffer");
  hipError_t e = sgk::launch_tip(c, q, tip);
  return e == hipSuccess ? SG_OK : hip_fail(c, e, "sg_tip_position");
}

sg_status sg_set_policy(sg_ctx* c, const sg_policy_arch* arch, const uint16_t* w, const float* b,
                        const float* log_std) {
  if (!c) return SG_E_INVAL;
  if (!arch || !w || !b || !log_std) return fail(c, SG_E_INVAL, "sg_set_policy: null argument");
  if (c->dtype != SG_F32) return fail(c, SG_E_UNSUPPORTED, "sg_set_policy: FP32 contexts only");
  const int h3 = policy_h3(arch);
  if (h3 < 0 || c->J > 7)
    return fail(c, SG_E_UNSUPPORTED,
                "sg_set_policy: supported are 256-128 tanh and 256-128-64 ELU networks with max_dof <= 7");
  if (h3 && c->prismatic) return fail(c, SG_E_UNSUPPORTED, "sg_set_policy: the 256-128-64 network needs revolute chains");
  const int W = 2 * c->J + 10, O = c->J + 1;
  const int dims[5] = {W, sgk::kH1, sgk::kH2, h3 ? h3 : O, O};
  const int nl = h3 ? 4 : 3;
  const uint16_t* Wl[4];
  const float* bl[4];
  size_t ow = 0, ob = 0;
  for (int l = 0; l < nl; ++l) {
    Wl[l] = w + ow;
    bl[l] = b + ob;
    ow += (size_t)dims[l + 1] * dims[l];
    ob += dims[l + 1];
  }
  std::vector<uint16_t> img;
  std::vector<float> bimg;
  if (h3) pack_policy_host<64>(W, O, Wl, bl, img, bimg);
  else pack_policy_host<0>(W, O, Wl, bl, img, bimg);
  hipError_t e = hipSuccess;
  // buffers sized for the larger network, so either can be set later
  if (!c->w_bf16) e = hipMalloc((void**)&c->w_bf16, (size_t)sgk::kWFragsMax * 16);
  if (e == hipSuccess && !c->bias) e = hipMalloc((void**)&c->bias, (size_t)sgk::kBiasMax * sizeof(float));
  if (e == hipSuccess && !c->log_std) e = hipMalloc((void**)&c->log_std, c->J * sizeof(float));
  if (e == hipSuccess) e = hipMemcpy(c->w_bf16, img.data(), img.size() * sizeof(uint16_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->bias, bimg.data(), bimg.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->log_std, log_std, c->J * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(c, e, "sg_set_policy");
  c->has_policy = 1;
  c->h1 = sgk::kH1;
  c->h2 = sgk::kH2;
  c->h3 = h3;
  c->pact = arch->act;
  return SG_OK;
}

sg_status sg_policy_forward(sg_ctx* c, const float* x, int32_t n, float* out) {
  if (!c) return SG_E_INVAL;
  if (!c->has_policy) return fail(c, SG_E_STATE, "sg_policy_forward: no policy set");
  if (!x || !out || n < 1 || !aligned(x) || !aligned(out))
    return fail(c, SG_E_INVAL, "sg_policy_forward: bad buffer or n");
  hipError_t e = sgk::launch_policy_forward(c, x, n, out);
  return e == hipSuccess ? SG_OK : hip_fail(c, e, "sg_policy_forward");
}

sg_status sg_rollout(sg_ctx* c, int32_t T, const sg_rollout_bufs* b) {
  if (!c) return SG_E_INVAL;
  if (c->dtype != SG_F32) return fail(c, SG_E_UNSUPPORTED, "sg_rollout: FP32 contexts only");
  if (!c->has_policy) return fail(c, SG_E_STATE, "sg_rollout: no policy set");
  if (!b || T < 1 || T > 4096) return fail(c, SG_E_INVAL, "sg_rollout: T must be in 1..4096");
  if (!b->obs || !b->act || !b->logp || !b->rew || !b->done || !b->val || !b->adv || !b->ret)
    return fail(c, SG_E_INVAL, "sg_rollout: null buffer");
  if (!aligned(b->obs) || !aligned(b->act) || !aligned(b->logp) || !aligned(b->rew) || !aligned(b->val) ||
      !aligned(b->adv) || !aligned(b->ret))
    return fail(c, SG_E_INVAL, "sg_rollout: misaligned buffer");
  hipError_t e = sgk::launch_rollout(c, T, b);
  return e == hipSuccess ? SG_OK : hip_fail(c, e, "sg_rollout");
}

sg_status sg_gae(sg_ctx* c, int32_t T, int32_t n, const float* rew, const float* val, const uint8_t* done, float gamma,
                 float lam, float* adv, float* ret) {
  if (!c) return SG_E_INVAL;
  if (T < 1 || n < 1 || !rew || !val || !done || !adv || !ret) return fail(c, SG_E_INVAL, "sg_gae: bad argument");
  hipError_t e = sgk::launch_gae(c->stream, T, n, rew, val, done, gamma, lam, adv, ret);
  return e == hipSuccess ? SG_OK : hip_fail(c, e, "sg_gae");
}

}  // extern "C"
