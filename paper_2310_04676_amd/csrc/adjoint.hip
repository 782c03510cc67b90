// Differentiation of an open-loop rollout: loss L_e = sum_t |tip(q_{t+1}) -
// goal_t| (the negated path-following / reaching reward, paper Sec. IV) of
// T control steps from the context's current state with given actions,
// and its gradients with respect to every action and every link mass.
//
// One kernel, one env per lane, the chain in VGPRs and its parameters in LDS:
//   forward   T steps, the state (q, qd, progress) stored every K steps
//             (checkpoints, [T/K][2J+1][N]);
//   reverse   segment by segment from the last: the segment's K steps are
//             recomputed from its checkpoint, keeping each substep's
//             starting state and acceleration in a tape [K S][3J][N] (plus
//             the post-step state and episode flags per step), then walked
//             backwards:
//             tip-distance gradient, hard stops, semi-implicit Euler, the
//             implicit forward-dynamics rule (an ABA solve with zero
//             velocity and gravity gives lambda = (H + arm)^-1 qdd_bar, then
//             vjp_rnea), and the PD torque.
// Memory: checkpoints + one segment's tape instead of the full tape
// (T S 2J floats per env).
#include <map>
#include <mutex>

#include "adj.hpp"
#include "internal.hpp"

namespace sgk {

struct AdjArgs {
  EnvDev<float> E;
  int T, K;
  const float* act;    // [T][J][N]
  float* loss;         // [N]
  float* g_act;        // [T][J][N]
  float* g_mass;       // [J][N]
  float* ckpt;         // [nseg][2J][N] q, qd
  int* ckpt_prog;      // [nseg][N]
  float* tape;         // [K S][3J][N] substep starting states q, qd and accelerations qdd
  float* tend;         // [K][J][N] post-step state before any reset
  int* tinfo;          // [K][N] progress before the step | reset flag << 30
};

template <int J, int M>
__global__ void __launch_bounds__(64) k_adjoint(AdjArgs A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const EnvDev<float>& E = A.E;
  float* sp = reinterpret_cast<float*>(smem_raw);
  const int e = blockIdx.x * 64 + threadIdx.x;
  const bool active = e < E.N;
  const int n = M == M_UNI ? J : (active ? E.nd[e] : 0);
  auto ps = ParOf<float, J, use_lds<float, J>(), M == M_PRI>::make(E, e, n, active, sp);
  if (!active) return;
  const size_t N = E.N;
  const int S = E.S;
  const float h = E.h;
  const float zero_g[3] = {0.f, 0.f, 0.f};
  const float tipl[3] = {E.tip[e], E.tip[N + e], E.tip[2 * N + e]};
  float q[J], qd[J], arm[J], half[J];
  load_state<float, J>(E, e, n, q, qd);
  int prog = E.prog[e];
  ps.fence();
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const Jp<float> p = ps.get(j);
    arm[j] = j < n ? h * p.kd + h * h * p.kp : 0.f;
    half[j] = j < n ? 0.5f * (p.hi - p.lo) : 0.f;
  }
  // one control step; optionally records substep states into the tape
  // (inlined: as a called function its captured arrays would live in
  // scratch memory)
  auto step = [&](int t, float* tp, float* te, int* ti) __attribute__((always_inline)) {
    float a[J];
#pragma unroll
    for (int j = 0; j < J; ++j) a[j] = j < n ? A.act[((size_t)t * E.J + j) * N + e] : 0.f;
    if (tp) {
      // physics() with the substep states recorded
      float qs[J], tau[J], qdd[J];
      ps.fence();
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const Jp<float> p = ps.get(j);
        qs[j] = j < n ? 0.5f * (p.hi + p.lo) + half[j] * clamp1(a[j]) : 0.f;
      }
      for (int s = 0; s < S; ++s) {
        float* dst = tp + (size_t)s * 3 * E.J * N;
        ps.fence();
#pragma unroll
        for (int j = 0; j < J; ++j) {
          if (j < n) {
            const Jp<float> p = ps.get(j);
            dst[(size_t)j * N + e] = q[j];
            dst[(size_t)(E.J + j) * N + e] = qd[j];
            tau[j] = p.kp * (qs[j] - q[j] - h * qd[j]) - p.kd * qd[j];
          } else {
            tau[j] = 0.f;
          }
        }
        aba_lwa<float, J>(ps, n, q, qd, tau, arm, E.g, qdd);
        ps.fence();
#pragma unroll
        for (int j = 0; j < J; ++j) {
          if (j < n) {
            const Jp<float> p = ps.get(j);
            dst[(size_t)(2 * E.J + j) * N + e] = qdd[j];
            qd[j] = qd[j] + h * qdd[j];
            q[j] = q[j] + h * qd[j];
            if (q[j] > p.hi) {
              q[j] = p.hi;
              if (qd[j] > 0.f) qd[j] = 0.f;
            } else if (q[j] < p.lo) {
              q[j] = p.lo;
              if (qd[j] < 0.f) qd[j] = 0.f;
            }
          }
        }
      }
    } else {
      physics<float, J>(E, ps, n, a, q, qd);
    }
    float tip[3], g[3];
    tip_fk<float, J>(ps, n, q, tipl, tip);
    goal_of(E, e, prog, g);
    const float dx = tip[0] - g[0], dy = tip[1] - g[1], dz = tip[2] - g[2];
    const float dist = sqrtf(dx * dx + dy * dy + dz * dz);
    if (te) {
#pragma unroll
      for (int j = 0; j < J; ++j)
        if (j < n) te[(size_t)j * N + e] = q[j];
    }
    const int pre = prog;
    prog = prog + 1;
    bool reset = false;
    if (E.ep_len > 0 && prog >= E.ep_len) {
      reset = true;
#pragma unroll
      for (int j = 0; j < J; ++j) {
        if (j < n) {
          q[j] = E.par[((size_t)P_Q0 * E.J + j) * N + e];
          qd[j] = 0.f;
        }
      }
      prog = 0;
    }
    if (ti) ti[e] = pre | (reset ? (1 << 30) : 0);
    return dist;
  };
  const int nseg = (A.T + A.K - 1) / A.K;
  // forward with checkpoints
  float L = 0.f;
  for (int t = 0; t < A.T; ++t) {
    if (t % A.K == 0) {
      float* c = A.ckpt + (size_t)(t / A.K) * 2 * E.J * N;
#pragma unroll
      for (int j = 0; j < J; ++j) {
        if (j < n) {
          c[(size_t)j * N + e] = q[j];
          c[(size_t)(E.J + j) * N + e] = qd[j];
        }
      }
      A.ckpt_prog[(size_t)(t / A.K) * N + e] = prog;
    }
    L += step(t, nullptr, nullptr, nullptr);
  }
  A.loss[e] = L;
  // reverse
  float qb[J], qdb[J], gm[J];
#pragma unroll
  for (int j = 0; j < J; ++j) qb[j] = qdb[j] = gm[j] = 0.f;
  for (int sg = nseg - 1; sg >= 0; --sg) {
    const int t0 = sg * A.K, t1 = min(A.T, t0 + A.K);
    const float* c = A.ckpt + (size_t)sg * 2 * E.J * N;
#pragma unroll
    for (int j = 0; j < J; ++j) {
      q[j] = j < n ? c[(size_t)j * N + e] : 0.f;
      qd[j] = j < n ? c[(size_t)(E.J + j) * N + e] : 0.f;
    }
    prog = A.ckpt_prog[(size_t)sg * N + e];
    for (int t = t0; t < t1; ++t)
      step(t, A.tape + (size_t)(t - t0) * S * 3 * E.J * N, A.tend + (size_t)(t - t0) * E.J * N,
           A.tinfo + (size_t)(t - t0) * N);
    for (int t = t1 - 1; t >= t0; --t) {
      const int info = A.tinfo[(size_t)(t - t0) * N + e];
      if (info >> 30) {
#pragma unroll
        for (int j = 0; j < J; ++j) qb[j] = qdb[j] = 0.f;
      }
      // tip-distance gradient at the post-step state
      float qe[J];
      const float* te = A.tend + (size_t)(t - t0) * E.J * N;
#pragma unroll
      for (int j = 0; j < J; ++j) qe[j] = j < n ? te[(size_t)j * N + e] : 0.f;
      {
        float tip[3], g[3];
        tip_fk<float, J>(ps, n, qe, tipl, tip);
        goal_of(E, e, info & ((1 << 30) - 1), g);
        float d[3] = {tip[0] - g[0], tip[1] - g[1], tip[2] - g[2]};
        const float dist = sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        const float inv = dist > 0.f ? 1.f / dist : 0.f;
        d[0] *= inv; d[1] *= inv; d[2] *= inv;
        tip_vjp<float, J>(ps, n, qe, tipl, d, qb);
      }
      float a[J], qsb[J];
#pragma unroll
      for (int j = 0; j < J; ++j) {
        a[j] = j < n ? A.act[((size_t)t * E.J + j) * N + e] : 0.f;
        qsb[j] = 0.f;
      }
      for (int s = S - 1; s >= 0; --s) {
        // the substep's state and the accelerations the recomputation found
        const float* src = A.tape + ((size_t)(t - t0) * S + s) * 3 * E.J * N;
        float q0[J], qd0[J], qdd[J], qddb[J], lam[J], zero[J], gq[J], gqd[J];
#pragma unroll
        for (int j = 0; j < J; ++j) {
          q0[j] = j < n ? src[(size_t)j * N + e] : 0.f;
          qd0[j] = j < n ? src[(size_t)(E.J + j) * N + e] : 0.f;
          qdd[j] = j < n ? src[(size_t)(2 * E.J + j) * N + e] : 0.f;
          zero[j] = 0.f;
          gq[j] = gqd[j] = 0.f;
        }
        ps.fence();
#pragma unroll
        for (int j = 0; j < J; ++j) {
          if (j < n) {
            const Jp<float> p = ps.get(j);
            const float qd1 = qd0[j] + h * qdd[j];
            const float q1 = q0[j] + h * qd1;
            float qbj = qb[j], qdbj = qdb[j];
            if (q1 > p.hi) {
              qbj = 0.f;
              if (qd1 > 0.f) qdbj = 0.f;
            } else if (q1 < p.lo) {
              qbj = 0.f;
              if (qd1 < 0.f) qdbj = 0.f;
            }
            qdbj += h * qbj;
            qb[j] = qbj;
            qdb[j] = qdbj;
            qddb[j] = h * qdbj;
          } else {
            qddb[j] = 0.f;
          }
        }
        aba<float, J, true>(ps, n, q0, zero, qddb, arm, zero_g, lam);
        vjp_rnea<float, J>(ps, n, q0, qd0, qdd, lam, E.g, gq, gqd, gm);
        ps.fence();
#pragma unroll
        for (int j = 0; j < J; ++j) {
          if (j < n) {
            const Jp<float> p = ps.get(j);
            qb[j] = qb[j] - gq[j] - p.kp * lam[j];
            qdb[j] = qdb[j] - gqd[j] - (p.kp * h + p.kd) * lam[j];
            qsb[j] += p.kp * lam[j];
          }
        }
      }
#pragma unroll
      for (int j = 0; j < J; ++j)
        if (j < E.J)
          A.g_act[((size_t)t * E.J + j) * N + e] = (j < n && a[j] > -1.f && a[j] < 1.f) ? half[j] * qsb[j] : 0.f;
    }
  }
  // vjp_rnea accumulated +d(lam . ID)/dm; the loss sees its negative
#pragma unroll
  for (int j = 0; j < J; ++j)
    if (j < E.J) A.g_mass[(size_t)j * N + e] = j < n ? -gm[j] : 0.f;
}

template <int J, int M> static hipError_t adjoint_j(const sg_ctx* c, const AdjArgs& A) {
  constexpr size_t lds = use_lds<float, J>() ? par_lds_bytes<float, J>() : 0;
  hipError_t e = lds_limit((const void*)k_adjoint<J, M>, lds);
  if (e != hipSuccess) return e;
  k_adjoint<J, M><<<dim3((c->N + 63) / 64), 64, lds, c->stream>>>(A);
  return hipGetLastError();
}

hipError_t launch_adjoint(const sg_ctx* c, int T, int K, const float* act, float* loss, float* g_act, float* g_mass,
                          float* ws) {
  AdjArgs A;
  A.E = env_view<float>(c);
  A.T = T; A.K = K; A.act = act; A.loss = loss; A.g_act = g_act; A.g_mass = g_mass;
  const size_t N = c->N, J2 = 2 * (size_t)c->J, J3 = 3 * (size_t)c->J, nseg = (T + K - 1) / K;
  A.ckpt = ws;
  A.ckpt_prog = reinterpret_cast<int*>(ws + nseg * J2 * N);
  A.tape = ws + nseg * (J2 + 1) * N;
  A.tend = A.tape + (size_t)K * c->S * J3 * N;
  A.tinfo = reinterpret_cast<int*>(A.tend + (size_t)K * c->J * N);
  if (c->prismatic) return c->J <= 4 ? adjoint_j<4, M_PRI>(c, A) : adjoint_j<7, M_PRI>(c, A);
  return c->J <= 4 ? adjoint_j<4, M_GEN>(c, A) : adjoint_j<7, M_GEN>(c, A);
}

size_t adjoint_ws_floats(const sg_ctx* c, int T, int K) {
  const size_t N = c->N, J2 = 2 * (size_t)c->J, J3 = 3 * (size_t)c->J, nseg = (T + K - 1) / K;
  return nseg * (J2 + 1) * N + (size_t)K * c->S * J3 * N + (size_t)K * c->J * N + (size_t)K * N;
}

// Rescale every inertial parameter of each link to new masses m [J][N]
// (geometry fixed).
template <typename T>
__global__ void __launch_bounds__(256) k_set_masses(T* __restrict__ par, int J, int N, const int* __restrict__ nd,
                                                    const T* __restrict__ m) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= J * N) return;
  const int j = i / N, e = i % N;
  if (j >= nd[e]) return;
  const size_t fs = (size_t)J * N;
  const T old = par[P_M * fs + i];
  const T s = m[i] / old;
  const int f[10] = {P_M, P_HX, P_HY, P_HZ, P_IXX, P_IYY, P_IZZ, P_IXY, P_IXZ, P_IYZ};
  for (int k = 0; k < 10; ++k) par[f[k] * fs + i] *= s;
}

hipError_t launch_set_masses(sg_ctx* c, const void* m) {
  const int n = c->J * c->N;
  if (c->dtype == SG_F64)
    k_set_masses<double><<<(n + 255) / 256, 256, 0, c->stream>>>((double*)c->par, c->J, c->N, c->nd, (const double*)m);
  else
    k_set_masses<float><<<(n + 255) / 256, 256, 0, c->stream>>>((float*)c->par, c->J, c->N, c->nd, (const float*)m);
  return hipGetLastError();
}

// Fixed workspace of sg_adjoint_static: 16 MiB of device memory per GPU,
// held until the process ends. Host code never passes the array's name to a
// kernel (on the host it is a stand-in, not a device address): it takes the
// address hipGetSymbolAddress returns for the device, once per device.
constexpr size_t kAdjStaticFloats = (size_t)4 << 20;
static __device__ __align__(256) float scratch[kAdjStaticFloats];

// This device's copy of scratch (dev current while the address is taken).
static hipError_t scratch_ptr(int dev, float** out) {
  static std::mutex mu;
  static std::map<int, float*> addr;
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(dev);
  if (it != addr.end()) {
    *out = it->second;
    return hipSuccess;
  }
  int cur = 0;
  hipError_t e = hipGetDevice(&cur);
  if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
  float* ptr = nullptr;
  if (e == hipSuccess) e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
  if (cur != dev) {
    const hipError_t e2 = hipSetDevice(cur);
    if (e == hipSuccess) e = e2;
  }
  if (e != hipSuccess) return e;
  addr[dev] = ptr;
  *out = ptr;
  return hipSuccess;
}

}  // namespace sgk

using namespace sgk;

extern "C" {

sg_status sg_adjoint(sg_ctx* c, int32_t T, int32_t K, const float* actions, float* loss, float* g_act,
                     float* g_mass) {
  if (!c) return SG_E_INVAL;
  if (c->dtype != SG_F32 || c->J > 7 || c->task == SG_TASK_TRACK) {
    c->err = "sg_adjoint: FP32 reaching or path-following contexts with max_dof <= 7 only";
    return SG_E_UNSUPPORTED;
  }
  if (T < 1 || K < 1 || K > T || !actions || !loss || !g_act || !g_mass) {
    c->err = "sg_adjoint: need 1 <= K <= T and non-null buffers";
    return SG_E_INVAL;
  }
  const size_t need = adjoint_ws_floats(c, T, K);
  hipError_t e = hipSuccess;
  if (need > c->adj_ws_floats) {
    e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess && c->adj_ws) e = hipFree(c->adj_ws);
    c->adj_ws = nullptr;
    c->adj_ws_floats = 0;
    if (e == hipSuccess) e = hipMalloc((void**)&c->adj_ws, need * sizeof(float));
    if (e == hipSuccess) c->adj_ws_floats = need;
  }
  if (e == hipSuccess) e = launch_adjoint(c, T, K, actions, loss, g_act, g_mass, c->adj_ws);
  if (e != hipSuccess) {
    c->err = std::string("sg_adjoint: ") + hipGetErrorString(e);
    return SG_E_HIP;
  }
  return SG_OK;
}

sg_status sg_adjoint_static(sg_ctx* c, int32_t T, int32_t K, const float* actions, float* loss, float* g_act,
                            float* g_mass) {
  if (!c) return SG_E_INVAL;
  if (c->dtype != SG_F32 || c->J > 7 || c->task == SG_TASK_TRACK) {
    c->err = "sg_adjoint_static: FP32 reaching or path-following contexts with max_dof <= 7 only";
    return SG_E_UNSUPPORTED;
  }
  if (T < 1 || K < 1 || K > T || !actions || !loss || !g_act || !g_mass) {
    c->err = "sg_adjoint_static: need 1 <= K <= T and non-null buffers";
    return SG_E_INVAL;
  }
  const size_t need = adjoint_ws_floats(c, T, K);
  if (need > kAdjStaticFloats) {
    c->err = "sg_adjoint_static: workspace of " + std::to_string(need * sizeof(float)) +
             " bytes exceeds the fixed " + std::to_string(kAdjStaticFloats * sizeof(float)) +
             " bytes (use sg_adjoint, or fewer envs, steps or a smaller K)";
    return SG_E_INVAL;
  }
  float* ws = nullptr;
  hipError_t e = scratch_ptr(c->device, &ws);
  if (e == hipSuccess) e = launch_adjoint(c, T, K, actions, loss, g_act, g_mass, ws);
  if (e != hipSuccess) {
    c->err = std::string("sg_adjoint_static: ") + hipGetErrorString(e);
    return SG_E_HIP;
  }
  return SG_OK;
}

int64_t sg_adjoint_workspace_bytes(const sg_ctx* c, int32_t T, int32_t K) {
  if (!c || T < 1 || K < 1 || K > T) return -1;
  return (int64_t)(adjoint_ws_floats(c, T, K) * sizeof(float));
}

sg_status sg_set_link_masses(sg_ctx* c, const void* masses) {
  if (!c) return SG_E_INVAL;
  if (!masses) {
    c->err = "sg_set_link_masses: null buffer";
    return SG_E_INVAL;
  }
  hipError_t e = launch_set_masses(c, masses);
  if (e != hipSuccess) {
    c->err = std::string("sg_set_link_masses: ") + hipGetErrorString(e);
    return SG_E_HIP;
  }
  return SG_OK;
}

}  // extern "C"
