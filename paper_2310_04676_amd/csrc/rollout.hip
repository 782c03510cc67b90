// Learning-side kernels: the fused T-step rollout (policy on the matrix
// cores, exploration noise, environment step), the policy alone, and the
// GAE backward scan.
#include "internal.hpp"
#include "mlp.hpp"

namespace sgk {

constexpr int kWave = 64;
constexpr int kXMax = 32;  // observation width padded to the first layer's K

// LDS layout of the rollout kernel (bytes): weight image, bias image,
// staged inputs, outputs, link parameters
// With a wave team, the Table II network's image does not fit beside the
// team's exchange: its layer-1 fragments (16 KB) are then read from the
// global image (L2) instead of LDS.
template <int H3, bool TEAM> constexpr bool w1_global() { return TEAM && H3 > 0; }
template <int H3, bool TEAM = false> constexpr size_t lds_w_bytes() {
  return (size_t)(PolicyShape<H3>::kWFrags - (w1_global<H3, TEAM>() ? kW1Frags : 0)) * 16;
}
template <int H3> constexpr size_t lds_bias_bytes() { return (size_t)PolicyShape<H3>::kBias * 4; }
constexpr size_t kLdsX = 256 * 16;
constexpr size_t kLdsO = (size_t)kWave * kOut * 4;
template <int J> constexpr size_t lds_par_bytes() { return (size_t)P_NSTAGE * J * kWave * 4; }
template <int H3, bool TEAM = false> constexpr size_t policy_lds_bytes() {
  return lds_w_bytes<H3, TEAM>() + lds_bias_bytes<H3>() + kLdsX + kLdsO;
}
// ... plus, with a wave team, the links the helper waves hand back (the
// published state reuses the staged-input area, idle during the physics),
// plus the exploration noise the helper waves draw one step ahead: two
// step-parity slots of one float4 per Philox block and lane
constexpr int kNoiseBlocks = 2;  // Philox blocks of four normals: chains of up to 7 joints
constexpr size_t kLdsEps = (size_t)2 * kNoiseBlocks * kWave * 16;
template <int J, int H3, bool TEAM = false> constexpr size_t rollout_lds_bytes() {
  return policy_lds_bytes<H3, TEAM>() + lds_par_bytes<J>() + (TEAM ? team_lds_bytes(J) : 0) + kLdsEps;
}
constexpr size_t kLdsMax = 160 * 1024;
static_assert(rollout_lds_bytes<7, 64>() <= kLdsMax, "the Table II network's rollout fits the LDS");
static_assert(rollout_lds_bytes<7, 0, true>() <= kLdsMax, "the 7-joint team rollout fits the LDS");
static_assert(rollout_lds_bytes<7, 64, true>() <= kLdsMax, "the Table II network's 7-joint team rollout fits the LDS");
static_assert((size_t)team_state_slots(7) * 64 * 16 <= kLdsX, "the team state fits the staged-input area");
// a wave team where its exchange fits next to the weight image
template <int J, int H3> constexpr bool team_fits() { return J >= 4 && rollout_lds_bytes<J, H3, true>() <= kLdsMax; }

struct RollArgs {
  EnvDev<float> E;
  const uint4* wimg;
  const float* bias;
  const float* log_std;
  int T;
  uint64_t seed;
  float* obs;
  float* act;
  float* logp;
  float* rew;
  uint8_t* done;
  float* val;
};

// GAE for env e: one lane walks t = T-1 .. 0; each step reads one
// coalesced row of rew / val / done and writes one row of adv / ret.
// delta_t = r_t + gamma V_{t+1} (1 - d_t) - V_t with r_t += gamma V_t on a
// time-out; A_t = delta_t + gamma lam (1 - d_t) A_{t+1}; R_t = A_t + V_t.
// The rows of kGaeChunk steps are loaded before the chunk's recursion runs,
// so the loads overlap instead of each waiting on the last.
constexpr int kGaeChunk = 16;
constexpr int kGaeBlock = 64;
__device__ __forceinline__ void gae_env(int T, int n, int e, const float* __restrict__ rew,
                                        const float* __restrict__ val, const uint8_t* __restrict__ done,
                                        float gamma, float lam, float* __restrict__ adv, float* __restrict__ ret) {
  float A = 0.f;
  float vnext = val[(size_t)T * n + e];
  for (int t1 = T; t1 > 0; t1 -= kGaeChunk) {
    const int t0 = t1 > kGaeChunk ? t1 - kGaeChunk : 0;  // this chunk: t0 .. t1-1
    float rr[kGaeChunk], vv[kGaeChunk];
    uint8_t dd[kGaeChunk];
#pragma unroll
    for (int k = 0; k < kGaeChunk; ++k) {
      const int t = t0 + k;
      if (t < t1) {
        const size_t i = (size_t)t * n + e;
        rr[k] = rew[i];
        vv[k] = val[i];
        dd[k] = done[i];
      }
    }
#pragma unroll
    for (int k = kGaeChunk - 1; k >= 0; --k) {
      const int t = t0 + k;
      if (t < t1) {
        const size_t i = (size_t)t * n + e;
        const uint8_t d = dd[k];
        const float v = vv[k];
        const float nd = (d & DONE_ENDED) ? 0.f : 1.f;
        const float r = rr[k] + ((d & DONE_TIMEOUT) ? gamma * v : 0.f);
        const float delta = r + gamma * vnext * nd - v;
        A = delta + gamma * lam * nd * A;
        adv[i] = A;
        ret[i] = A + v;
        vnext = v;
      }
    }
  }
}

// the weight image from fragment f0 on (f0 = kW1Frags: layer 1 stays in
// the global image) and the bias image
template <int H3>
__device__ __forceinline__ void fill_weights(uint4* sw, float* sb, const uint4* __restrict__ wimg,
                                             const float* __restrict__ bias, int tid, int nthreads, int f0 = 0) {
  for (int i = tid; i < PolicyShape<H3>::kWFrags - f0; i += nthreads) sw[i] = wimg[f0 + i];
  for (int i = tid; i < PolicyShape<H3>::kBias; i += nthreads) sb[i] = bias[i];
}

// One workgroup = 64 envs and four waves, for all T steps: weights and the
// envs' link parameters are staged in LDS once, the chain state stays in
// wave 0's VGPRs (one env per lane). Every step the four waves run the
// policy on the matrix cores, one 16-env tile each (they share the LDS
// weight image; each wave alone on its SIMD), then wave 0 samples the
// action, advances the physics and writes the step's rollout rows. With
// TEAM the other three waves share every substep's solve as a wave team
// (aba_lwa_team); without it they wait at the next step's barrier.
// Control flow around the barriers is uniform per wave: wave 0 runs the
// physics for all of its lanes (lanes past N on zeros, storing nothing).
constexpr int kRollWaves = 4;
static_assert(kRollWaves == kTeam, "the rollout's waves form one team");
template <int J, int M, int H3, int ACT, bool TEAM>
__global__ void __launch_bounds__(kWave * kRollWaves) k_rollout(RollArgs A) {
  extern __shared__ __align__(16) unsigned char lds[];
  constexpr bool kW1G = w1_global<H3, TEAM>();
  constexpr size_t kLdsW = lds_w_bytes<H3, TEAM>(), kLdsBias = lds_bias_bytes<H3>();
  uint4* s_w = reinterpret_cast<uint4*>(lds);
  float* s_b = reinterpret_cast<float*>(lds + kLdsW);
  uint4* s_x = reinterpret_cast<uint4*>(lds + kLdsW + kLdsBias);
  float* s_o = reinterpret_cast<float*>(lds + kLdsW + kLdsBias + kLdsX);
  float* s_p = reinterpret_cast<float*>(lds + kLdsW + kLdsBias + kLdsX + kLdsO);
  const EnvDev<float>& E = A.E;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & (kWave - 1);
  const bool phys = wave == 0;  // the wave that owns the envs' state
  const int e = blockIdx.x * kWave + lane;
  const bool active = phys && e < E.N;
  const int n = M == M_UNI ? J : (active ? E.nd[e] : 0);
  // the team: state published in the staged-input area, links after the
  // link parameters; a helper's joint count is its lane's env's
  const TeamLds team{reinterpret_cast<float4*>(s_x),
                     reinterpret_cast<float4*>(lds + kLdsW + kLdsBias + kLdsX + kLdsO + lds_par_bytes<J>()), wave,
                     lane};
  const int n_help = M == M_UNI ? J : (e < E.N ? E.nd[e] : 0);
  const int Wd = 2 * E.J + 10;
  const size_t N = E.N;
  const uint64_t step0 = read_counter(E);
  // the noise slots: [2 step parities][noise block][64 lanes]; helper wave w
  // (1 .. blocks) draws block w-1 of the next step's normals
  float4* s_eps = reinterpret_cast<float4*>(lds + rollout_lds_bytes<J, H3, TEAM>() - kLdsEps);
  constexpr int kNb = (J + 3) / 4;
  static_assert(kNb <= kNoiseBlocks && kNb < kRollWaves, "one helper wave per noise block");
  auto draw = [&](int t) __attribute__((always_inline)) {
    if (wave >= 1 && wave <= kNb) {
      float v[4];
      normals4(A.seed, (uint32_t)e, step0 + (uint64_t)t, (uint32_t)(wave - 1), v);
      s_eps[((t & 1) * kNoiseBlocks + wave - 1) * kWave + lane] = make_float4(v[0], v[1], v[2], v[3]);
    }
  };

  fill_weights<H3>(s_w, s_b, A.wimg, A.bias, threadIdx.x, kWave * kRollWaves, kW1G ? kW1Frags : 0);
  if (phys) stage_chain<float, J>(E, e, active ? n : 0, lane, s_p);
  draw(0);
  __syncthreads();
  LdsPar<float, J, M == M_PRI> ps{s_p, lane};
  float lstd[J], sig[J];
  float lp_const = 0.f;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    lstd[j] = j < n ? A.log_std[j] : 0.f;
    sig[j] = __expf(lstd[j]);
    if (j < n) lp_const -= lstd[j] + 0.91893853320467274f;
  }

  float q[J], qd[J], x[kXMax];
#pragma unroll
  for (int j = 0; j < J; ++j) { q[j] = 0.f; qd[j] = 0.f; }
  int prog = 0;
  if (active) {
    load_state<float, J>(E, e, n, q, qd);
    prog = E.prog[e];
    const float tipl[3] = {E.tip[e], E.tip[N + e], E.tip[2 * N + e]};
    float tip[3], g[3];
    tip_fk<float, J>(ps, n, q, tipl, tip);
    goal_of(E, e, prog, g);
    obs_regs<float, J, kXMax>(E, n, q, qd, tip, g, x);
    for (int k = 0; k < Wd; ++k) A.obs[(size_t)k * N + e] = x[k];
  } else {
#pragma unroll
    for (int k = 0; k < kXMax; ++k) x[k] = 0.f;
  }
  __syncthreads();

  for (int t = 0; t <= A.T; ++t) {
    if (phys) stage_input(s_x, lane, x, Wd);
    __syncthreads();
    mlp_wave<H3, ACT, 1, kW1G>(s_w, s_b, s_x, s_o, lane, wave, A.wimg);
    __syncthreads();
    if (!phys) {
      if (t == A.T) break;
      // the next step's noise: with a team once the first substep's links
      // are handed back (wave 0 is in that substep's inward pass), else now
      if constexpr (TEAM) physics_help<J>(E, ps, n_help, team, [&] { draw(t + 1); });
      else draw(t + 1);
      continue;
    }
    float mu[J];
#pragma unroll
    for (int j = 0; j < J; ++j) mu[j] = s_o[lane * kOut + j];
    const float V = s_o[lane * kOut + E.J];
    if (active) A.val[(size_t)t * N + e] = V;
    if (t == A.T) break;
    float a[J];
#pragma unroll
    for (int j = 0; j < J; ++j) a[j] = 0.f;
    if (active) {
      // this step's normals, drawn by the helper waves (the same values as
      // normals(): block b holds joints 4b .. 4b+3; joints >= n take 0)
      float eps[J];
#pragma unroll
      for (int b = 0; b < kNb; ++b) {
        const float4 v = s_eps[((t & 1) * kNoiseBlocks + b) * kWave + lane];
        const float w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (4 * b + k < J) eps[4 * b + k] = 4 * b + k < n ? w4[k] : 0.f;
      }
      float lp = lp_const;
#pragma unroll
      for (int j = 0; j < J; ++j) {
        a[j] = j < n ? mu[j] + sig[j] * eps[j] : 0.f;
        lp -= 0.5f * eps[j] * eps[j];
        if (j < E.J) A.act[((size_t)t * E.J + j) * N + e] = a[j];
      }
      A.logp[(size_t)t * N + e] = lp;
    }
    if constexpr (TEAM) {
      physics<float, J, LdsPar<float, J, M == M_PRI>, true>(E, ps, n, a, q, qd, team);
    } else {
      if (active) physics<float, J>(E, ps, n, a, q, qd);
    }
    if (!active) continue;
    float r, tip[3], g[3];
    const uint8_t d = post_step<float, J>(E, e, n, ps, q, qd, prog, &r, A.obs + (size_t)(t + 1) * Wd * N, tip, g,
                                          step0 + (uint64_t)t);
    obs_regs<float, J, kXMax>(E, n, q, qd, tip, g, x);
    A.rew[(size_t)t * N + e] = r;
    A.done[(size_t)t * N + e] = d;
  }
  if (active) store_state<float, J>(E, e, n, q, qd, prog);
  // every wave read the counter before the loop's first barrier
  if (threadIdx.x == 0) advance_counter(E, step0, true);
}

// The policy alone on n inputs x [W][n] -> out [J+1][n].
template <int H3, int ACT>
__global__ void __launch_bounds__(kWave) k_policy(const uint4* __restrict__ wimg, const float* __restrict__ bias,
                                                  int Wd, int n_out, int n, const float* __restrict__ xin,
                                                  float* __restrict__ out) {
  extern __shared__ __align__(16) unsigned char lds[];
  constexpr size_t kLdsW = lds_w_bytes<H3>(), kLdsBias = lds_bias_bytes<H3>();
  uint4* s_w = reinterpret_cast<uint4*>(lds);
  float* s_b = reinterpret_cast<float*>(lds + kLdsW);
  uint4* s_x = reinterpret_cast<uint4*>(lds + kLdsW + kLdsBias);
  float* s_o = reinterpret_cast<float*>(lds + kLdsW + kLdsBias + kLdsX);
  const int lane = threadIdx.x;
  const int e = blockIdx.x * kWave + lane;
  fill_weights<H3>(s_w, s_b, wimg, bias, lane, kWave);
  float x[kXMax];
#pragma unroll
  for (int k = 0; k < kXMax; ++k) x[k] = (e < n && k < Wd) ? xin[(size_t)k * n + e] : 0.f;
  stage_input(s_x, lane, x, Wd);
  __syncthreads();
  mlp_wave<H3, ACT>(s_w, s_b, s_x, s_o, lane);
  __syncthreads();
  if (e < n)
    for (int i = 0; i < n_out; ++i) out[(size_t)i * n + e] = s_o[lane * kOut + i];
}

// The GAE scan (after each rollout, and sg_gae): one lane per env.
__global__ void __launch_bounds__(kGaeBlock) k_gae(int T, int n, const float* __restrict__ rew,
                                                   const float* __restrict__ val, const uint8_t* __restrict__ done,
                                                   float gamma, float lam, float* __restrict__ adv,
                                                   float* __restrict__ ret) {
  const int e = blockIdx.x * kGaeBlock + threadIdx.x;
  if (e < n) gae_env(T, n, e, rew, val, done, gamma, lam, adv, ret);
}

hipError_t launch_gae(hipStream_t s, int T, int n, const float* rew, const float* val, const uint8_t* done,
                      float gamma, float lam, float* adv, float* ret) {
  k_gae<<<dim3((n + kGaeBlock - 1) / kGaeBlock), kGaeBlock, 0, s>>>(T, n, rew, val, done, gamma, lam, adv, ret);
  return hipGetLastError();
}

template <int H3, int ACT> static hipError_t policy_forward_t(const sg_ctx* c, const float* x, int n, float* out) {
  const size_t lds = policy_lds_bytes<H3>();
  hipError_t e = lds_limit((const void*)k_policy<H3, ACT>, lds);
  if (e != hipSuccess) return e;
  k_policy<H3, ACT><<<dim3((n + kWave - 1) / kWave), kWave, lds, c->stream>>>(
      reinterpret_cast<const uint4*>(c->w_bf16), c->bias, 2 * c->J + 10, c->J + 1, n, x, out);
  return hipGetLastError();
}

hipError_t launch_policy_forward(const sg_ctx* c, const float* x, int n, float* out) {
  if (c->h3) return policy_forward_t<64, PACT_ELU>(c, x, n, out);
  return policy_forward_t<0, PACT_TANH>(c, x, n, out);
}

template <int J, int M, int H3 = 0, int ACT = PACT_TANH>
static hipError_t rollout_j(sg_ctx* c, int T, const sg_rollout_bufs* b) {
  constexpr bool kFits = team_fits<J, H3>();
  const bool team = kFits && c->team != 1;  // the team or auto: one block per compute unit either way
  const size_t lds = team ? rollout_lds_bytes<J, H3, kFits>() : rollout_lds_bytes<J, H3>();
  const void* fn = team ? (const void*)k_rollout<J, M, H3, ACT, kFits> : (const void*)k_rollout<J, M, H3, ACT, false>;
  hipError_t e = lds_limit(fn, lds);
  if (e != hipSuccess) return e;
  RollArgs A;
  A.E = env_view<float>(c);
  A.E.rng_add = (uint32_t)T;
  A.wimg = reinterpret_cast<const uint4*>(c->w_bf16);
  A.bias = c->bias;
  A.log_std = c->log_std;
  A.T = T;
  A.seed = c->seed;
  A.obs = b->obs; A.act = b->act; A.logp = b->logp; A.rew = b->rew; A.done = b->done; A.val = b->val;
  const dim3 grid((c->N + kWave - 1) / kWave);
  if (team) k_rollout<J, M, H3, ACT, kFits><<<grid, kWave * kRollWaves, lds, c->stream>>>(A);
  else k_rollout<J, M, H3, ACT, false><<<grid, kWave * kRollWaves, lds, c->stream>>>(A);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_gae(c->stream, T, c->N, b->rew, b->val, b->done, b->gamma, b->lam, b->adv, b->ret);
}

hipError_t launch_rollout(sg_ctx* c, int T, const sg_rollout_bufs* b) {
  const bool u = c->uniform;
  if (c->h3) {
    // the Table II network (256-128-64 ELU): revolute chains of up to 7 joints
    return u && c->J == 7 ? rollout_j<7, M_UNI, 64, PACT_ELU>(c, T, b) : rollout_j<7, M_GEN, 64, PACT_ELU>(c, T, b);
  }
  if (c->prismatic) return c->J <= 4 ? rollout_j<4, M_PRI>(c, T, b) : rollout_j<7, M_PRI>(c, T, b);
  switch (dof_bucket(c->J)) {
    case 1: return rollout_j<1, M_UNI>(c, T, b);
    case 2: return u ? rollout_j<2, M_UNI>(c, T, b) : rollout_j<2, M_GEN>(c, T, b);
    case 4: return u ? rollout_j<4, M_UNI>(c, T, b) : rollout_j<4, M_GEN>(c, T, b);
    default: return u ? rollout_j<7, M_UNI>(c, T, b) : rollout_j<7, M_GEN>(c, T, b);
  }
}

}  // namespace sgk
