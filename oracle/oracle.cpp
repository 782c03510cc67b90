// Test infrastructure: the FP64 CPU oracle's C interface. Only tests/, the
// smoke check and the CPU-baseline leg of the benchmark may load or run this
// library; the product path never does. It shares no code with the HIP
// library: it is written independently from the paper and from Featherstone's
// textbook, and is checked against closed forms, invariants and brute force.
//
// Array layout matches the synthetic-input generator: structure of arrays,
// [field][joint][env] for per-joint data and [field][env] for per-env data,
// all float64 (done flags uint8, progress int32).
#include <cmath>
#include <cstdint>
#include <cstring>

#include "chain.hpp"
#include "counted.hpp"
#include "env.hpp"
#include "rl.hpp"

#ifdef _OPENMP
#include <omp.h>
#endif

using namespace ora;

extern "C" {

typedef struct {
  int32_t n_env, max_dof;
  const int32_t* n_dof;   // [N]
  const double* axis;     // [3][J][N] unit joint axis (parent = child coords)
  const double* offset;   // [3][J][N] joint origin in the parent link frame
  const double* com;      // [3][J][N] centre of mass in the link frame
  const double* mass;     // [J][N]
  const double* inertia;  // [6][J][N] xx yy zz xy xz yz about the centre of mass
  const double* kp;       // [J][N]
  const double* kd;       // [J][N]
  const double* q_lo;     // [J][N]
  const double* q_hi;     // [J][N]
  const double* q0;       // [J][N] reset position
  const double* tip;      // [3][N] tool tip in the last link frame
  double dt;
  int32_t substeps;
  double gravity[3];
  const int32_t* joint_type;  // [J][N] 0 revolute, 1 prismatic; null: all revolute
} ora_robot;

typedef struct {
  int32_t task, n_waypoints, dwell, ep_len;
  const double* target;     // [3][N] (reach; tracking: the first episode's centre)
  const double* waypoints;  // [K][3][N]
  double trk_sigma, trk_offset, trk_reset_std, trk_centre[3];  // tracking task
  int32_t chains;           // chains per env (multi-tool reaching); <= 1: one
  // per-episode re-randomisation (reach, path; one chain per env): waypoints
  // then hold n_banks sets [n_banks K][3][N]
  int32_t rerand, n_banks;
  double rand_centre[3], rand_half;
} ora_task;

typedef struct {
  int32_t n_layers;         // 3 or 4 (2 or 3 hidden layers)
  int32_t dims[5];          // n_in, hidden sizes, n_out
  const double* W[4];       // row-major [n_out][n_in] per layer
  const double* b[4];
  const double* log_std;    // [n_out - 1]
  int32_t act;              // hidden activation: 0 tanh, 1 ELU
} ora_policy;

}  // extern "C"

namespace {

template <class T> Chain<T> load_chain(const ora_robot* r, int e) {
  const int N = r->n_env, J = r->max_dof;
  Chain<T> ch;
  ch.n = r->n_dof[e];
  for (int j = 0; j < ch.n; ++j) {
    Link<T>& l = ch.L[j];
    l.type = r->joint_type ? r->joint_type[j * N + e] : kRevolute;
    auto at = [&](const double* a, int f) { return T(a[(f * J + j) * N + e]); };
    l.axis = v3(at(r->axis, 0), at(r->axis, 1), at(r->axis, 2));
    l.offset = v3(at(r->offset, 0), at(r->offset, 1), at(r->offset, 2));
    l.com = v3(at(r->com, 0), at(r->com, 1), at(r->com, 2));
    l.mass = at(r->mass, 0);
    T xx = at(r->inertia, 0), yy = at(r->inertia, 1), zz = at(r->inertia, 2);
    T xy = at(r->inertia, 3), xz = at(r->inertia, 4), yz = at(r->inertia, 5);
    l.Ic.m[0][0] = xx; l.Ic.m[0][1] = xy; l.Ic.m[0][2] = xz;
    l.Ic.m[1][0] = xy; l.Ic.m[1][1] = yy; l.Ic.m[1][2] = yz;
    l.Ic.m[2][0] = xz; l.Ic.m[2][1] = yz; l.Ic.m[2][2] = zz;
    finalize_link(l);
  }
  ch.tip = v3(T(r->tip[0 * N + e]), T(r->tip[1 * N + e]), T(r->tip[2 * N + e]));
  ch.grav = v3(T(r->gravity[0]), T(r->gravity[1]), T(r->gravity[2]));
  return ch;
}

template <class T> Drive<T> load_drive(const ora_robot* r, int e) {
  const int N = r->n_env;
  Drive<T> d;
  for (int j = 0; j < r->n_dof[e]; ++j) {
    d.kp[j] = T(r->kp[j * N + e]);
    d.kd[j] = T(r->kd[j * N + e]);
    d.lo[j] = T(r->q_lo[j * N + e]);
    d.hi[j] = T(r->q_hi[j * N + e]);
    d.q0[j] = T(r->q0[j * N + e]);
  }
  return d;
}

TaskSpec load_taskspec(const ora_task* t, int N) {
  TaskSpec s;
  s.task = t->task;
  s.n_waypoints = t->n_waypoints;
  s.dwell = t->dwell;
  s.ep_len = t->ep_len;
  s.trk_sigma = t->trk_sigma;
  s.trk_offset = t->trk_offset;
  s.trk_reset_std = t->trk_reset_std;
  for (int k = 0; k < 3; ++k) s.trk_centre[k] = t->trk_centre[k];
  s.chains = t->chains > 1 ? t->chains : 1;
  s.rerand = t->rerand;
  s.n_banks = t->n_banks > 1 ? t->n_banks : 1;
  for (int k = 0; k < 3; ++k) s.rand_centre[k] = t->rand_centre[k];
  s.rand_half = t->rand_half;
  s.wp_all = t->waypoints;
  s.N = N;
  return s;
}

template <class T> EnvGoal<T> load_goal(const ora_task* t, int N, int e) {
  EnvGoal<T> g;
  if (t->target) g.target = v3(T(t->target[0 * N + e]), T(t->target[1 * N + e]), T(t->target[2 * N + e]));
  else g.target = v3(T(0.0), T(0.0), T(0.0));
  for (int k = 0; k < t->n_waypoints && t->waypoints; ++k) {
    const double* w = t->waypoints + (size_t)k * 3 * N;
    g.wp[k] = v3(T(w[0 * N + e]), T(w[1 * N + e]), T(w[2 * N + e]));
  }
  return g;
}

// Gather per-joint SoA [J][N] column of env e into a dense vector.
void gather(const double* a, int /*J*/, int N, int e, int n, double* out) {
  for (int j = 0; j < n; ++j) out[j] = a[j * N + e];
}
void scatter(double* a, int /*J*/, int N, int e, int n, const double* in) {
  for (int j = 0; j < n; ++j) a[j * N + e] = in[j];
}

}  // namespace

extern "C" {

int ora_max_dof() { return kMaxDof; }

int ora_fk(const ora_robot* r, const double* q, double* tip) {
  const int N = r->n_env, J = r->max_dof;
  for (int e = 0; e < N; ++e) {
    Chain<double> ch = load_chain<double>(r, e);
    double qe[kMaxDof];
    gather(q, J, N, e, ch.n, qe);
    Pose<double> P;
    forward_kinematics(ch, qe, P);
    tip[0 * N + e] = P.tip.x;
    tip[1 * N + e] = P.tip.y;
    tip[2 * N + e] = P.tip.z;
  }
  return 0;
}

// World position of every link's centre of mass and joint origin, and the
// link orientations: com_w [3][J][N], joint_w [3][J][N], R_w [9][J][N].
int ora_fk_links(const ora_robot* r, const double* q, double* com_w, double* joint_w, double* R_w) {
  const int N = r->n_env, J = r->max_dof;
  for (int e = 0; e < N; ++e) {
    Chain<double> ch = load_chain<double>(r, e);
    double qe[kMaxDof];
    gather(q, J, N, e, ch.n, qe);
    Pose<double> P;
    forward_kinematics(ch, qe, P);
    for (int j = 0; j < ch.n; ++j) {
      V3<double> c = P.p[j] + mul(P.R[j], ch.L[j].com);
      com_w[(0 * J + j) * N + e] = c.x;
      com_w[(1 * J + j) * N + e] = c.y;
      com_w[(2 * J + j) * N + e] = c.z;
      joint_w[(0 * J + j) * N + e] = P.p[j].x;
      joint_w[(1 * J + j) * N + e] = P.p[j].y;
      joint_w[(2 * J + j) * N + e] = P.p[j].z;
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) R_w[((a * 3 + b) * J + j) * N + e] = P.R[j].m[a][b];
    }
  }
  return 0;
}

int ora_rnea(const ora_robot* r, const double* q, const double* qd, const double* qdd, double* tau) {
  const int N = r->n_env, J = r->max_dof;
  for (int e = 0; e < N; ++e) {
    Chain<double> ch = load_chain<double>(r, e);
    double qe[kMaxDof], qde[kMaxDof], qdde[kMaxDof], te[kMaxDof];
    gather(q, J, N, e, ch.n, qe);
    gather(qd, J, N, e, ch.n, qde);
    gather(qdd, J, N, e, ch.n, qdde);
    rnea(ch, qe, qde, qdde, te);
    scatter(tau, J, N, e, ch.n, te);
  }
  return 0;
}

// H: [N][J][J] row-major per env (top-left n x n used).
int ora_crba(const ora_robot* r, const double* q, double* H) {
  const int N = r->n_env, J = r->max_dof;
  for (int e = 0; e < N; ++e) {
    Chain<double> ch = load_chain<double>(r, e);
    double qe[kMaxDof], He[kMaxDof * kMaxDof];
    gather(q, J, N, e, ch.n, qe);
    crba(ch, qe, He);
    for (int i = 0; i < J * J; ++i) H[(size_t)e * J * J + i] = 0.0;
    for (int i = 0; i < ch.n; ++i)
      for (int j = 0; j < ch.n; ++j) H[(size_t)e * J * J + i * J + j] = He[i * ch.n + j];
  }
  return 0;
}

// arm may be null (zero armature).
int ora_aba(const ora_robot* r, const double* q, const double* qd, const double* tau, const double* arm,
            double* qdd) {
  const int N = r->n_env, J = r->max_dof;
  for (int e = 0; e < N; ++e) {
    Chain<double> ch = load_chain<double>(r, e);
    double qe[kMaxDof], qde[kMaxDof], te[kMaxDof], ae[kMaxDof] = {0}, oe[kMaxDof];
    gather(q, J, N, e, ch.n, qe);
    gather(qd, J, N, e, ch.n, qde);
    gather(tau, J, N, e, ch.n, te);
    if (arm) gather(arm, J, N, e, ch.n, ae);
    aba(ch, qe, qde, te, ae, oe);
    scatter(qdd, J, N, e, ch.n, oe);
  }
  return 0;
}

// Second route to the same answer: qdd = (H + diag(arm))^{-1} (tau - C),
// C = RNEA(q, qd, 0). Returns the number of envs whose matrix failed Cholesky.
int ora_fd_crba(const ora_robot* r, const double* q, const double* qd, const double* tau, const double* arm,
                double* qdd) {
  const int N = r->n_env, J = r->max_dof;
  int bad = 0;
  for (int e = 0; e < N; ++e) {
    Chain<double> ch = load_chain<double>(r, e);
    const int n = ch.n;
    double qe[kMaxDof], qde[kMaxDof], te[kMaxDof], ae[kMaxDof] = {0}, zero[kMaxDof] = {0};
    double C[kMaxDof], H[kMaxDof * kMaxDof], rhs[kMaxDof], x[kMaxDof];
    gather(q, J, N, e, n, qe);
    gather(qd, J, N, e, n, qde);
    gather(tau, J, N, e, n, te);
    if (arm) gather(arm, J, N, e, n, ae);
    rnea(ch, qe, qde, zero, C);
    crba(ch, qe, H);
    for (int i = 0; i < n; ++i) {
      H[i * n + i] += ae[i];
      rhs[i] = te[i] - C[i];
    }
    if (!cholesky_solve(n, H, rhs, x)) {
      ++bad;
      for (int i = 0; i < n; ++i) x[i] = NAN;
    }
    scatter(qdd, J, N, e, n, x);
  }
  return bad;
}

// Observation of the given state, obs [2J+10][N].
// Tracking task: goal_state [9][N] = (goal, goal velocity, centre), updated
// in place; draws from Philox counter (seed; env, step).
static Track<double> load_track(const double* gs, int N, int e) {
  Track<double> tr;
  tr.g = v3(gs[0 * N + e], gs[1 * N + e], gs[2 * N + e]);
  tr.gd = v3(gs[3 * N + e], gs[4 * N + e], gs[5 * N + e]);
  tr.gc = v3(gs[6 * N + e], gs[7 * N + e], gs[8 * N + e]);
  return tr;
}
static void store_track(double* gs, int N, int e, const Track<double>& tr) {
  const double v[9] = {tr.g.x, tr.g.y, tr.g.z, tr.gd.x, tr.gd.y, tr.gd.z, tr.gc.x, tr.gc.y, tr.gc.z};
  for (int k = 0; k < 9; ++k) gs[k * N + e] = v[k];
}
// Re-randomised reach / path tasks: goal_state [3][N] = the episode's target
// (reach), [1][N] = the index of its waypoint set (path).
static Rerand<double> load_rerand(const TaskSpec& ts, const double* gs, int N, int e) {
  Rerand<double> rr;
  if (ts.task == kTaskReach) rr.target = v3(gs[0 * N + e], gs[1 * N + e], gs[2 * N + e]);
  else rr.bank = (int)gs[e];
  return rr;
}
static void store_rerand(const TaskSpec& ts, double* gs, int N, int e, const Rerand<double>& rr) {
  if (ts.task == kTaskReach) {
    gs[0 * N + e] = rr.target.x; gs[1 * N + e] = rr.target.y; gs[2 * N + e] = rr.target.z;
  } else {
    gs[e] = (double)rr.bank;
  }
}

int ora_observe(const ora_robot* r, const ora_task* t, const double* q, const double* qd, const int32_t* progress,
                double* obs, const double* goal_state) {
  const int N = r->n_env, J = r->max_dof, W = 2 * J + 10;
  TaskSpec ts = load_taskspec(t, r->n_env);
  for (int e = 0; e < N; ++e) {
    Chain<double> ch = load_chain<double>(r, e);
    EnvGoal<double> g = load_goal<double>(t, N, e);
    double qe[kMaxDof], qde[kMaxDof], oe[64];
    gather(q, J, N, e, ch.n, qe);
    gather(qd, J, N, e, ch.n, qde);
    Track<double> tr;
    if (ts.task == kTaskTrack) tr = load_track(goal_state, N, e);
    if (ts.rerand) apply_rerand(ts, load_rerand(ts, goal_state, N, e), e, g);
    observe(ch, J, ts, g, qe, qde, progress[e], oe, ts.task == kTaskTrack ? &tr : nullptr);
    for (int w = 0; w < W; ++w) obs[w * N + e] = oe[w];
  }
  return 0;
}

// One control step for envs [e0, e1). State (q, qd, progress) updated in
// place. qdd_log [S][J][N] may be null. Uses OpenMP over envs if compiled
// with it and n_threads > 1.
int ora_step(const ora_robot* r, const ora_task* t, const double* action, double* q, double* qd,
             int32_t* progress, double* reward, uint8_t* done, double* obs, double* qdd_log, int e0, int e1,
             int n_threads, double* goal_state, uint64_t seed, uint64_t step) {
  const int N = r->n_env, J = r->max_dof, W = 2 * J + 10, S = r->substeps;
  TaskSpec ts = load_taskspec(t, r->n_env);
  (void)n_threads;
  if (ts.chains > 1) {
    // multi-chain envs: chains [k C, (k + 1) C) form env k
    const int C = ts.chains;
    if (e0 % C || e1 % C || N % C) return -1;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(n_threads > 0 ? n_threads : 1)
#endif
    for (int k = e0 / C; k < e1 / C; ++k) {
      Chain<double> ch[kMaxChains];
      Drive<double> dr[kMaxChains];
      EnvGoal<double> g[kMaxChains];
      Track<double> tr[kMaxChains];
      double qe[kMaxChains][kMaxDof], qde[kMaxChains][kMaxDof], ae[kMaxChains][kMaxDof], oe[kMaxChains][64];
      double* qp[kMaxChains];
      double* qdp[kMaxChains];
      double* op[kMaxChains];
      const double* ap[kMaxChains];
      uint32_t lane[kMaxChains];
      for (int c = 0; c < C; ++c) {
        const int e = k * C + c;
        ch[c] = load_chain<double>(r, e);
        dr[c] = load_drive<double>(r, e);
        g[c] = load_goal<double>(t, N, e);
        if (ts.task == kTaskTrack) tr[c] = load_track(goal_state, N, e);
        gather(q, J, N, e, ch[c].n, qe[c]);
        gather(qd, J, N, e, ch[c].n, qde[c]);
        gather(action, J, N, e, ch[c].n, ae[c]);
        qp[c] = qe[c]; qdp[c] = qde[c]; op[c] = oe[c]; ap[c] = ae[c];
        lane[c] = (uint32_t)e;
      }
      int prog = progress[k * C];
      double rew;
      const uint8_t d = group_step(C, ch, dr, r->dt, S, J, ts, g, ap, qp, qdp, &prog, &rew, op,
                                   ts.task == kTaskTrack ? tr : nullptr, seed, lane, step);
      for (int c = 0; c < C; ++c) {
        const int e = k * C + c;
        if (ts.task == kTaskTrack) store_track(goal_state, N, e, tr[c]);
        scatter(q, J, N, e, ch[c].n, qe[c]);
        scatter(qd, J, N, e, ch[c].n, qde[c]);
        progress[e] = prog;
        reward[e] = rew;
        done[e] = d;
        for (int w = 0; w < W; ++w) obs[w * N + e] = oe[c][w];
      }
    }
    return 0;
  }
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(n_threads > 0 ? n_threads : 1)
#endif
  for (int e = e0; e < e1; ++e) {
    Chain<double> ch = load_chain<double>(r, e);
    Drive<double> dr = load_drive<double>(r, e);
    EnvGoal<double> g = load_goal<double>(t, N, e);
    const int n = ch.n;
    double qe[kMaxDof], qde[kMaxDof], ae[kMaxDof], oe[64], rew, qlog[64 * kMaxDof];
    gather(q, J, N, e, n, qe);
    gather(qd, J, N, e, n, qde);
    gather(action, J, N, e, n, ae);
    int prog = progress[e];
    Track<double> tr;
    Track<double>* trp = nullptr;
    if (ts.task == kTaskTrack) {
      tr = load_track(goal_state, N, e);
      trp = &tr;
    }
    Rerand<double> rr;
    Rerand<double>* rrp = nullptr;
    if (ts.rerand) {
      rr = load_rerand(ts, goal_state, N, e);
      apply_rerand(ts, rr, e, g);
      rrp = &rr;
    }
    uint8_t d = env_step(ch, dr, r->dt, S, J, ts, g, ae, qe, qde, &prog, &rew, oe, qdd_log ? qlog : nullptr, trp,
                         seed, (uint32_t)e, step, rrp);
    if (trp) store_track(goal_state, N, e, tr);
    if (rrp) store_rerand(ts, goal_state, N, e, rr);
    scatter(q, J, N, e, n, qe);
    scatter(qd, J, N, e, n, qde);
    progress[e] = prog;
    reward[e] = rew;
    done[e] = d;
    for (int w = 0; w < W; ++w) obs[w * N + e] = oe[w];
    if (qdd_log)
      for (int s = 0; s < S; ++s)
        for (int j = 0; j < n; ++j) qdd_log[((size_t)s * J + j) * N + e] = qlog[s * n + j];
  }
  return 0;
}

// Exact operation count of one control step of env e (physics substeps,
// kinematics, reward, observation), and separately of the physics substeps
// alone. counts: [add, mul, div, sqrt, trans] x 2 (step, physics).
int ora_opcount_step(const ora_robot* r, const ora_task* t, int e, const double* action, long long* counts) {
  const int N = r->n_env, J = r->max_dof;
  TaskSpec ts = load_taskspec(t, r->n_env);
  Chain<Counted> ch = load_chain<Counted>(r, e);
  Drive<Counted> dr = load_drive<Counted>(r, e);
  EnvGoal<Counted> g = load_goal<Counted>(t, N, e);
  const int n = ch.n;
  Counted qe[kMaxDof], qde[kMaxDof], ae[kMaxDof], oe[64], rew;
  for (int j = 0; j < n; ++j) {
    qe[j] = Counted(r->q0[j * N + e]);
    qde[j] = Counted(0.0);
    ae[j] = Counted(action[j * N + e]);
  }
  int prog = 0;
  tally() = OpTally();
  env_step(ch, dr, Counted(r->dt), r->substeps, J, ts, g, ae, qe, qde, &prog, &rew, oe, (Counted*)nullptr);
  OpTally all = tally();
  for (int j = 0; j < n; ++j) {
    qe[j] = Counted(r->q0[j * N + e]);
    qde[j] = Counted(0.0);
  }
  tally() = OpTally();
  physics_step(ch, dr, Counted(r->dt), r->substeps, ae, qe, qde, (Counted*)nullptr);
  OpTally phys = tally();
  counts[0] = all.add; counts[1] = all.mul; counts[2] = all.div; counts[3] = all.sqrt; counts[4] = all.trans;
  counts[5] = phys.add; counts[6] = phys.mul; counts[7] = phys.div; counts[8] = phys.sqrt; counts[9] = phys.trans;
  return 0;
}

// Operation tallies of single spatial-algebra primitives applied once to
// Counted operands, in the order: dot, cross, 3x3 matrix-vector, 3x3
// matrix-matrix, motion transform, transposed force transform, motion cross
// product, force cross product, spatial inertia times vector, motion-force
// pairing, inertia congruence, inertia sum, axis rotation. out: [13][5] =
// add, mul, div, sqrt, trans per primitive. Returns the primitive count.
int ora_opcount_primitives(long long* out) {
  auto V = [](double a, double b, double c) { return v3(Counted(a), Counted(b), Counted(c)); };
  M3<Counted> A, B;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      A.m[i][j] = Counted(0.1 * (i + 1) + 0.01 * j);
      B.m[i][j] = Counted(0.2 * (j + 1) - 0.03 * i);
    }
  const V3<Counted> a = V(0.3, -0.2, 0.9), b = V(-0.4, 0.5, 0.1);
  const SV<Counted> m = {a, b}, f = {b, a};
  PX<Counted> X;
  X.E = A;
  X.r = b;
  SI<Counted> I = {A, B, A};
  int k = 0;
  auto rec = [&](auto&& fn) {
    tally() = OpTally();
    fn();
    const OpTally t = tally();
    long long* o = out + 5 * k++;
    o[0] = t.add; o[1] = t.mul; o[2] = t.div; o[3] = t.sqrt; o[4] = t.trans;
  };
  rec([&] { (void)dot(a, b); });
  rec([&] { (void)cross(a, b); });
  rec([&] { (void)mul(A, a); });
  rec([&] { (void)mul(A, B); });
  rec([&] { (void)xform_motion(X, m); });
  rec([&] { (void)xform_force_T(X, f); });
  rec([&] { (void)crm(m, f); });
  rec([&] { (void)crf(m, f); });
  rec([&] { (void)mul(I, m); });
  rec([&] { (void)sdot(m, f); });
  rec([&] { (void)congruence(X, I); });
  rec([&] { (void)add(I, I); });
  rec([&] { (void)axis_rotation(a, Counted(0.7)); });
  tally() = OpTally();
  return k;
}

// ---- learning side -------------------------------------------------------

void ora_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
  Philox4 c = {{ctr[0], ctr[1], ctr[2], ctr[3]}};
  Philox4 o = philox4x32_10(c, key[0], key[1]);
  for (int i = 0; i < 4; ++i) out[i] = o.v[i];
}

// eps [n][N] for envs 0..N-1 at one step.
void ora_noise(uint64_t seed, uint64_t step, int n, int N, double* eps) {
  double tmp[kMaxDof];
  for (int e = 0; e < N; ++e) {
    gaussian_noise(seed, (uint32_t)e, step, n, tmp);
    for (int j = 0; j < n; ++j) eps[j * N + e] = tmp[j];
  }
}

double ora_round_bf16(double x) { return round_bf16(x); }

// Policy forward on B inputs: x [n_in][B], out [n_out][B] (SoA).
int ora_mlp_forward(const ora_policy* p, const double* x, double* out, int B, int emulate) {
  MlpLayer L[4];
  const int nl = p->n_layers;
  for (int l = 0; l < nl; ++l) L[l] = {p->dims[l], p->dims[l + 1], p->W[l], p->b[l]};
  const int n_in = p->dims[0], n_out = p->dims[nl];
  double xe[1024], oe[1024], sa[1024], sb[1024];
  for (int e = 0; e < B; ++e) {
    for (int k = 0; k < n_in; ++k) xe[k] = x[k * B + e];
    mlp_forward(L, nl, xe, oe, emulate != 0, sa, sb, p->act);
    for (int i = 0; i < n_out; ++i) out[i * B + e] = oe[i];
  }
  return 0;
}

int ora_gae(int T, int N, const double* rew, const double* val_, const uint8_t* done, double gamma, double lam,
            double* adv, double* ret) {
  for (int e = 0; e < N; ++e) gae_env(T, N, e, rew, val_, done, gamma, lam, adv, ret);
  return 0;
}

// Whole rollout of T steps for envs [e0, e1) (paper Sec. III: the policy acts,
// the simulator steps, rewards are stored; then GAE). Buffers (SoA):
// obs [T+1][W][N] with obs[0] the input observation; act [T][J][N] (the
// sampled pre-clamp action); logp, rew [T][N]; done [T][N]; val [T+1][N];
// adv, ret [T][N]. State q, qd, progress updated in place. Noise uses step
// counter step0 + t.
int ora_rollout(const ora_robot* r, const ora_task* t, const ora_policy* p, int T, uint64_t seed, uint64_t step0,
                double gamma, double lam, int emulate, double* q, double* qd, int32_t* progress, double* obs,
                double* act, double* logp, double* rew, uint8_t* done, double* val_, double* adv, double* ret,
                int e0, int e1, int n_threads, double* goal_state) {
  const int N = r->n_env, J = r->max_dof, W = 2 * J + 10, S = r->substeps;
  TaskSpec ts = load_taskspec(t, r->n_env);
  MlpLayer L[4];
  const int nl = p->n_layers, hact = p->act;
  for (int l = 0; l < nl; ++l) L[l] = {p->dims[l], p->dims[l + 1], p->W[l], p->b[l]};
  const double half_log_2pi = 0.91893853320467274178032973640562;
  if (ts.chains > 1) {
    // multi-chain envs: each chain acts on its own observation with the
    // shared policy; the env's reward and episode are shared (group_step)
    const int C = ts.chains;
    if (e0 % C || e1 % C || N % C) return -1;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads > 0 ? n_threads : 1)
#endif
    for (int kk = e0 / C; kk < e1 / C; ++kk) {
      Chain<double> ch[kMaxChains];
      Drive<double> dr[kMaxChains];
      EnvGoal<double> g[kMaxChains];
      Track<double> tr[kMaxChains];
      double qe[kMaxChains][kMaxDof], qde[kMaxChains][kMaxDof], a[kMaxChains][kMaxDof], x[kMaxChains][64];
      double o[64], sa[1024], sb[1024], eps[kMaxDof];
      double* qp[kMaxChains];
      double* qdp[kMaxChains];
      double* xp[kMaxChains];
      const double* ap[kMaxChains];
      uint32_t lane[kMaxChains];
      for (int c = 0; c < C; ++c) {
        const int e = kk * C + c;
        ch[c] = load_chain<double>(r, e);
        dr[c] = load_drive<double>(r, e);
        g[c] = load_goal<double>(t, N, e);
        if (ts.task == kTaskTrack) tr[c] = load_track(goal_state, N, e);
        gather(q, J, N, e, ch[c].n, qe[c]);
        gather(qd, J, N, e, ch[c].n, qde[c]);
        for (int w = 0; w < W; ++w) x[c][w] = obs[(size_t)w * N + e];
        qp[c] = qe[c]; qdp[c] = qde[c]; xp[c] = x[c]; ap[c] = a[c];
        lane[c] = (uint32_t)e;
      }
      int prog = progress[kk * C];
      for (int s = 0; s < T; ++s) {
        for (int c = 0; c < C; ++c) {
          const int e = kk * C + c, n = ch[c].n;
          mlp_forward(L, nl, x[c], o, emulate != 0, sa, sb, hact);
          gaussian_noise(seed, (uint32_t)e, step0 + (uint64_t)s, n, eps);
          double lp = 0.0;
          for (int j = 0; j < n; ++j) {
            const double sigma = std::exp(p->log_std[j]);
            a[c][j] = o[j] + sigma * eps[j];
            lp += -0.5 * eps[j] * eps[j] - p->log_std[j] - half_log_2pi;
            act[((size_t)s * J + j) * N + e] = a[c][j];
          }
          for (int j = n; j < J; ++j) act[((size_t)s * J + j) * N + e] = 0.0;
          val_[(size_t)s * N + e] = o[J];
          logp[(size_t)s * N + e] = lp;
        }
        double rw;
        const uint8_t d = group_step(C, ch, dr, r->dt, S, J, ts, g, ap, qp, qdp, &prog, &rw, xp,
                                     ts.task == kTaskTrack ? tr : nullptr, seed, lane, step0 + (uint64_t)s);
        for (int c = 0; c < C; ++c) {
          const int e = kk * C + c;
          rew[(size_t)s * N + e] = rw;
          done[(size_t)s * N + e] = d;
          for (int w = 0; w < W; ++w) obs[((size_t)(s + 1) * W + w) * N + e] = x[c][w];
        }
      }
      for (int c = 0; c < C; ++c) {
        const int e = kk * C + c;
        mlp_forward(L, nl, x[c], o, emulate != 0, sa, sb, hact);
        val_[(size_t)T * N + e] = o[J];
        if (ts.task == kTaskTrack) store_track(goal_state, N, e, tr[c]);
        scatter(q, J, N, e, ch[c].n, qe[c]);
        scatter(qd, J, N, e, ch[c].n, qde[c]);
        progress[e] = prog;
      }
    }
    for (int e = e0; e < e1; ++e) gae_env(T, N, e, rew, val_, done, gamma, lam, adv, ret);
    return 0;
  }
  (void)n_threads;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4) num_threads(n_threads > 0 ? n_threads : 1)
#endif
  for (int e = e0; e < e1; ++e) {
    Chain<double> ch = load_chain<double>(r, e);
    Drive<double> dr = load_drive<double>(r, e);
    EnvGoal<double> g = load_goal<double>(t, N, e);
    const int n = ch.n;
    double qe[kMaxDof], qde[kMaxDof], x[64], o[64], sa[1024], sb[1024], eps[kMaxDof], a[kMaxDof];
    gather(q, J, N, e, n, qe);
    gather(qd, J, N, e, n, qde);
    int prog = progress[e];
    Track<double> tr;
    Track<double>* trp = nullptr;
    if (ts.task == kTaskTrack) {
      tr = load_track(goal_state, N, e);
      trp = &tr;
    }
    Rerand<double> rr;
    Rerand<double>* rrp = nullptr;
    if (ts.rerand) {
      rr = load_rerand(ts, goal_state, N, e);
      apply_rerand(ts, rr, e, g);
      rrp = &rr;
    }
    for (int w = 0; w < W; ++w) x[w] = obs[(size_t)w * N + e];
    for (int s = 0; s < T; ++s) {
      mlp_forward(L, nl, x, o, emulate != 0, sa, sb, hact);
      gaussian_noise(seed, (uint32_t)e, step0 + (uint64_t)s, n, eps);
      double lp = 0.0;
      for (int j = 0; j < n; ++j) {
        double sigma = std::exp(p->log_std[j]);
        a[j] = o[j] + sigma * eps[j];
        lp += -0.5 * eps[j] * eps[j] - p->log_std[j] - half_log_2pi;
        act[((size_t)s * J + j) * N + e] = a[j];
      }
      for (int j = n; j < J; ++j) act[((size_t)s * J + j) * N + e] = 0.0;
      val_[(size_t)s * N + e] = o[J];
      logp[(size_t)s * N + e] = lp;
      double rw;
      uint8_t d = env_step(ch, dr, r->dt, S, J, ts, g, a, qe, qde, &prog, &rw, x, (double*)nullptr, trp, seed,
                           (uint32_t)e, step0 + (uint64_t)s, rrp);
      rew[(size_t)s * N + e] = rw;
      done[(size_t)s * N + e] = d;
      for (int w = 0; w < W; ++w) obs[((size_t)(s + 1) * W + w) * N + e] = x[w];
    }
    mlp_forward(L, nl, x, o, emulate != 0, sa, sb, hact);
    val_[(size_t)T * N + e] = o[J];
    if (trp) store_track(goal_state, N, e, tr);
    if (rrp) store_rerand(ts, goal_state, N, e, rr);
    scatter(q, J, N, e, n, qe);
    scatter(qd, J, N, e, n, qde);
    progress[e] = prog;
  }
  for (int e = e0; e < e1; ++e) gae_env(T, N, e, rew, val_, done, gamma, lam, adv, ret);
  return 0;
}

}  // extern "C"

// ---- learned surrogate ----------------------------------------------------
#include "surrogate.hpp"

extern "C" {

typedef struct {
  int32_t n_layers;
  const int32_t* dims;        // n_layers + 1
  const double* const* W;     // per layer [dims[l+1]][dims[l]]
  const double* const* b;     // per layer [dims[l+1]]
  const double* mu_x;         // [dims[0]] input normalisation
  const double* sd_x;
  const double* mu_y;         // [dims[L]] output normalisation
  const double* sd_y;
} ora_surrogate;

}  // extern "C"

namespace {

SurrogateNet make_net(const ora_surrogate* s) {
  SurrogateNet n;
  n.n_layers = s->n_layers;
  n.dims.assign(s->dims, s->dims + s->n_layers + 1);
  n.W.assign(s->W, s->W + s->n_layers);
  n.b.assign(s->b, s->b + s->n_layers);
  return n;
}

}  // namespace

extern "C" {

// Raw surrogate features of samples with robot env ids env[B]:
// x [3J + 10J][B] = q, qd, tau (J each), then per joint j the standard
// inertial parameters (m, m c, I about the link origin: xx yy zz xy xz yz).
int ora_surrogate_features(const ora_robot* r, const double* q, const double* qd, const double* tau,
                           const int32_t* env, int B, double* x) {
  const int J = r->max_dof;
  const int F = 13 * J;
  for (int s = 0; s < B; ++s) {
    const int e = env[s];
    Chain<double> ch = load_chain<double>(r, e);
    for (int f = 0; f < F; ++f) x[(size_t)f * B + s] = 0.0;
    for (int j = 0; j < ch.n; ++j) {
      x[(size_t)j * B + s] = q[(size_t)j * B + s];
      x[(size_t)(J + j) * B + s] = qd[(size_t)j * B + s];
      x[(size_t)(2 * J + j) * B + s] = tau[(size_t)j * B + s];
      const Link<double>& l = ch.L[j];
      const double m = l.mass;
      const V3<double> c = l.com;
      const double c2 = dot(c, c);
      const double p[10] = {m, m * c.x, m * c.y, m * c.z,
                            l.Ic.m[0][0] + m * (c2 - c.x * c.x), l.Ic.m[1][1] + m * (c2 - c.y * c.y),
                            l.Ic.m[2][2] + m * (c2 - c.z * c.z), l.Ic.m[0][1] - m * c.x * c.y,
                            l.Ic.m[0][2] - m * c.x * c.z, l.Ic.m[1][2] - m * c.y * c.z};
      for (int k = 0; k < 10; ++k) x[(size_t)(3 * J + 10 * j + k) * B + s] = p[k];
    }
  }
  return 0;
}

// Normalised forward: out [dims[L]][B] denormalised prediction. If
// out_norm is non-null it receives the normalised network output.
int ora_surrogate_forward(const ora_surrogate* s, const double* x_raw, int B, int emulate, double* out,
                          double* out_norm) {
  SurrogateNet net = make_net(s);
  const int F = net.dims[0], O = net.dims[net.n_layers];
  std::vector<double> x(F), y(O);
  std::vector<std::vector<double>> acts, pre;
  for (int b = 0; b < B; ++b) {
    for (int f = 0; f < F; ++f) x[f] = (x_raw[(size_t)f * B + b] - s->mu_x[f]) / s->sd_x[f];
    surrogate_forward(net, x.data(), emulate != 0, acts, pre, y.data());
    for (int i = 0; i < O; ++i) {
      if (out_norm) out_norm[(size_t)i * B + b] = y[i];
      out[(size_t)i * B + b] = y[i] * s->sd_y[i] + s->mu_y[i];
    }
  }
  return 0;
}

// Mean squared error on normalised targets and its gradients (concatenated
// per layer into gW [sum dims[l+1]*dims[l]], gb [sum dims[l+1]]). target
// [O][B] raw accelerations. Returns the loss.
double ora_surrogate_grad(const ora_surrogate* s, const double* x_raw, const double* target, int B, int emulate,
                          double* gW_all, double* gb_all) {
  SurrogateNet net = make_net(s);
  const int L = net.n_layers, F = net.dims[0], O = net.dims[L];
  std::vector<std::vector<double>> gW(L), gb(L);
  for (int l = 0; l < L; ++l) {
    gW[l].assign((size_t)net.dims[l + 1] * net.dims[l], 0.0);
    gb[l].assign(net.dims[l + 1], 0.0);
  }
  std::vector<double> x(F), y(O), dy(O);
  std::vector<std::vector<double>> acts, pre;
  double loss = 0.0;
  const double scale = 1.0 / ((double)B * O);
  for (int b = 0; b < B; ++b) {
    for (int f = 0; f < F; ++f) x[f] = (x_raw[(size_t)f * B + b] - s->mu_x[f]) / s->sd_x[f];
    surrogate_forward(net, x.data(), emulate != 0, acts, pre, y.data());
    for (int i = 0; i < O; ++i) {
      const double t = (target[(size_t)i * B + b] - s->mu_y[i]) / s->sd_y[i];
      const double d = y[i] - t;
      loss += d * d * scale;
      dy[i] = 2.0 * d * scale;
    }
    surrogate_backward(net, acts, pre, dy.data(), emulate != 0, gW, gb);
  }
  size_t ow = 0, ob = 0;
  for (int l = 0; l < L; ++l) {
    for (size_t i = 0; i < gW[l].size(); ++i) gW_all[ow + i] = gW[l][i];
    for (size_t i = 0; i < gb[l].size(); ++i) gb_all[ob + i] = gb[l][i];
    ow += gW[l].size();
    ob += gb[l].size();
  }
  return loss;
}

int ora_adam(int n, double* w, const double* g, double* m, double* v, double lr, double beta1, double beta2,
             double eps, int t) {
  adam_update(n, w, g, m, v, lr, beta1, beta2, eps, t);
  return 0;
}

// Residual check of a predicted acceleration: rel[e] = |RNEA(q, qd, qdd_hat)
// + arm qdd_hat - tau| / max(|tau|, 1e-3). arm may be null (zero).
int ora_residual(const ora_robot* r, const double* q, const double* qd, const double* tau, const double* qdd_hat,
                 const double* arm, double* rel) {
  const int N = r->n_env, J = r->max_dof;
  for (int e = 0; e < N; ++e) {
    Chain<double> ch = load_chain<double>(r, e);
    const int n = ch.n;
    double qe[kMaxDof], qde[kMaxDof], te[kMaxDof], ae[kMaxDof] = {0}, he[kMaxDof], id[kMaxDof];
    gather(q, J, N, e, n, qe);
    gather(qd, J, N, e, n, qde);
    gather(tau, J, N, e, n, te);
    gather(qdd_hat, J, N, e, n, he);
    if (arm) gather(arm, J, N, e, n, ae);
    rnea(ch, qe, qde, he, id);
    double rr = 0.0, tt = 0.0;
    for (int j = 0; j < n; ++j) {
      const double d = id[j] + ae[j] * he[j] - te[j];
      rr += d * d;
      tt += te[j] * te[j];
    }
    rel[e] = std::sqrt(rr) / std::max(std::sqrt(tt), 1e-3);
  }
  return 0;
}


// ---- PPO update (paper Sec. III "Policy learning and control") ----------
}  // extern "C"
#include "ppo.hpp"
extern "C" {

// cfg = {clip, c_v, c_e, max_norm, lr, beta1, beta2, adam_eps}
static PpoCfg ppo_cfg(const double* c) { return PpoCfg{c[0], c[1], c[2], c[3], c[4], c[5], c[6], c[7]}; }

// Network of the PPO calls: arch = {L, n_in, h_1 .. h_L, J, act} (L hidden
// layers, act 0 tanh / 1 ELU).
static PpoNet ppo_net(const int* arch) {
  const int L = arch[0];
  std::vector<int> hidden(arch + 2, arch + 2 + L);
  return PpoNet(arch[1], hidden, arch[2 + L], arch[3 + L]);
}

// Gradient of one minibatch (no clipping, no update); network arch as in
// ppo_net; x [n_in][B], a [J][B], logp_old, adv (already normalised), ret, v_old
// [B]. g [P] is overwritten; stats = {loss_pi, loss_v, entropy, approx_kl,
// clip_frac}. Returns the total loss.
double ora_ppo_grad(const int* arch, const double* p, const double* x, const double* a, const double* logp_old,
                    const double* adv, const double* ret, const double* v_old, int B, const double* cfg, int emulate,
                    double* g, double* stats) {
  const PpoNet net = ppo_net(arch);
  const PpoCfg c = ppo_cfg(cfg);
  std::vector<std::vector<double>> xs(B, std::vector<double>(net.n_in)), as(B, std::vector<double>(net.J));
  std::vector<PpoSample> mb(B);
  for (int r = 0; r < B; ++r) {
    for (int k = 0; k < net.n_in; ++k) xs[r][k] = x[(size_t)k * B + r];
    for (int j = 0; j < net.J; ++j) as[r][j] = a[(size_t)j * B + r];
    mb[r] = PpoSample{xs[r].data(), as[r].data(), logp_old[r], adv[r], ret[r], v_old[r]};
  }
  std::fill(g, g + net.size, 0.0);
  const PpoStats st = ppo_minibatch(net, p, mb, c, emulate != 0, g);
  stats[0] = st.loss_pi; stats[1] = st.loss_v; stats[2] = st.entropy; stats[3] = st.approx_kl;
  stats[4] = st.clip_frac;
  return ppo_loss(st, c);
}

// Advantage normalisation over n values.
void ora_ppo_normalise(int n, const double* adv, double* out) { normalise_adv(n, adv, out); }

// Global-norm gradient clipping in place; returns the norm before clipping.
double ora_clip_grad_norm(int n, double* g, double max_norm) { return clip_grad_norm(n, g, max_norm); }

// A whole update on rollout buffers of T steps x N envs (layouts of
// ora_rollout): advantages normalised over all T N samples, then for each
// epoch the samples perm[ep][.] (identity if perm is null) are cut into
// n_mb minibatches of T N / n_mb; each minibatch: gradient, norm clip,
// Adam step (t counts the steps taken so far, updated). p, m, v [P] in place.
// stats: the mean over minibatches of {loss_pi, loss_v, entropy, approx_kl,
// clip_frac}.
int ora_ppo_update(const int* arch, double* p, double* m, double* v, int* t, const double* obs, const double* act,
                   const double* logp, const double* adv, const double* ret, const double* val_, int T, int N,
                   const int* perm, int epochs, int n_mb, const double* cfg, int emulate, double* stats) {
  const PpoNet net = ppo_net(arch);
  const PpoCfg c = ppo_cfg(cfg);
  const int W = net.n_in, J = net.J, B = T * N, mbs = B / n_mb;
  if (mbs * n_mb != B) return -1;
  std::vector<double> an(B), xs((size_t)B * W), as((size_t)B * J);
  normalise_adv(B, adv, an.data());
  for (int s = 0; s < B; ++s) {
    const int tt = s / N, e = s % N;
    for (int k = 0; k < W; ++k) xs[(size_t)s * W + k] = obs[((size_t)tt * W + k) * N + e];
    for (int j = 0; j < J; ++j) as[(size_t)s * J + j] = act[((size_t)tt * J + j) * N + e];
  }
  std::vector<double> g(net.size);
  for (int k = 0; k < 5; ++k) stats[k] = 0;
  for (int ep = 0; ep < epochs; ++ep) {
    for (int k = 0; k < n_mb; ++k) {
      std::vector<PpoSample> mb(mbs);
      for (int r = 0; r < mbs; ++r) {
        const int s = perm ? perm[(size_t)ep * B + (size_t)k * mbs + r] : k * mbs + r;
        const int tt = s / N, e = s % N;
        mb[r] = PpoSample{&xs[(size_t)s * W], &as[(size_t)s * J], logp[(size_t)tt * N + e], an[s],
                          ret[(size_t)tt * N + e], val_[(size_t)tt * N + e]};
      }
      std::fill(g.begin(), g.end(), 0.0);
      const PpoStats st = ppo_minibatch(net, p, mb, c, emulate != 0, g.data());
      clip_grad_norm(net.size, g.data(), c.max_norm);
      *t += 1;
      adam_update(net.size, p, g.data(), m, v, c.lr, c.beta1, c.beta2, c.adam_eps, *t);
      const double w = 1.0 / (epochs * n_mb);
      stats[0] += st.loss_pi * w; stats[1] += st.loss_v * w; stats[2] += st.entropy * w;
      stats[3] += st.approx_kl * w; stats[4] += st.clip_frac * w;
    }
  }
  return 0;
}


// ---- adjoint of an open-loop rollout (differentiation row) ---------------
}  // extern "C"
#include "adjoint.hpp"
extern "C" {

// Loss L_e = sum_t |tip(q_{t+1}) - goal_t| of a T-step open-loop rollout per
// env, from (q0, qd0, progress0) with actions act [T][J][N]; mass_scale
// [J][N] (may be null) multiplies each link's mass and inertia. With
// want_grad: g_act [T][J][N] = dL/da and g_mass [J][N] = dL/dm (d/d of the
// scaled mass). Envs [0, N) over `threads` OpenMP threads.
int ora_adjoint(const ora_robot* r, const ora_task* t, int T, const double* act, const double* q0, const double* qd0,
                const int32_t* prog0, const double* mass_scale, int want_grad, double* loss, double* g_act,
                double* g_mass, int threads) {
  const int N = r->n_env, J = r->max_dof;
  const TaskSpec ts = load_taskspec(t, r->n_env);
#pragma omp parallel for schedule(static) num_threads(threads > 0 ? threads : 1)
  for (int e = 0; e < N; ++e) {
    Chain<double> ch = load_chain<double>(r, e);
    const int n = ch.n;
    if (mass_scale)
      for (int j = 0; j < n; ++j) scale_link_mass(ch.L[j], mass_scale[j * N + e]);
    Drive<double> dr = load_drive<double>(r, e);
    EnvGoal<double> g = load_goal<double>(t, N, e);
    std::vector<double> a((size_t)T * n);
    double qe[kMaxDof], qde[kMaxDof];
    for (int k = 0; k < T; ++k)
      for (int j = 0; j < n; ++j) a[(size_t)k * n + j] = act[((size_t)k * J + j) * N + e];
    for (int j = 0; j < n; ++j) {
      qe[j] = q0[j * N + e];
      qde[j] = qd0[j * N + e];
    }
    AdjointOut o = rollout_adjoint(ch, dr, r->dt, r->substeps, ts, g, T, a.data(), qe, qde, prog0 ? prog0[e] : 0,
                                   want_grad != 0);
    loss[e] = o.loss;
    if (want_grad) {
      for (int j = 0; j < J; ++j) {
        if (g_mass) g_mass[j * N + e] = j < n ? o.g_mass[j] : 0.0;
        for (int k = 0; k < T; ++k)
          if (g_act) g_act[((size_t)k * J + j) * N + e] = j < n ? o.g_act[(size_t)k * n + j] : 0.0;
      }
    }
  }
  return 0;
}

}  // extern "C"
