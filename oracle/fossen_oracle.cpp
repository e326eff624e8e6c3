/*
 * fossen_oracle.cpp -- FP64 CPU oracle for the batched Fossen 6-DOF step.
 *
 * TEST INFRASTRUCTURE ONLY.  It is loaded by the test-suite, by the package
 * smoke check and by the benchmark's CPU-baseline leg, and by nothing else.
 * The GPU library never links, loads or calls it, and the two share no code:
 * this file derives every matrix (allocation, mass, Coriolis, restoring) from
 * the raw preset numbers by itself.
 *
 * What it computes (MarineGym, Sec. II "Method", Eq. (1)):
 *
 *   tau = M_RB nu' + C_RB(nu) nu + g_RB(eta) + M_A nu' + C_A(nu) nu + D(nu) nu + g_A(eta)
 *
 * with eta the NED pose and nu = (u,v,w,p,q,r) the body-fixed velocity
 * (Sec. II, the definitions under Eq. (1)).  The paper defers every term to
 * Fossen's handbook; the standard forms used here are:
 *
 *   M_RB = [[m I, -m S(r_g)], [m S(r_g), I_g - m S(r_g)^2]],  M = M_RB + diag(M_A)
 *   C(nu) = [[0, -S(M11 v + M12 w)], [-S(M11 v + M12 w), -S(M21 v + M22 w)]]
 *           (the skew form of C_RB + C_A; C is linear in M)
 *   D(nu) nu = (D_L + D_Q |nu|) nu   (diagonal linear + quadratic damping)
 *   g = -[(W - B) k ; (W r_g - B r_b) x k],  k = R(q)^T e_3,  W = m g0
 *
 * Readings where the paper is silent (each is listed with its reason in the
 * design notes): the attitude is a Hamilton scalar-first unit quaternion q
 * (body -> NED) instead of Euler angles; the equation is integrated coupled
 * (M = M_RB + M_A on the left) by classical RK4 with q renormalised after each
 * substep only; the action of Eq. (3) is a throttle in [-1,1] (clamped) mapped
 * to thrust linearly or as a|a| times F_max, held over the substeps of one
 * control step, optionally through a first-order lag f' = (f_cmd - f)/tau_thr
 * that is part of the RK4 state; tau = B_alloc f with column i = [d_i; r_i x d_i].
 *
 * The algebra is dense and FP64: the mass matrix is rebuilt and solved by a
 * Cholesky factorisation in every right-hand side.  Everything is a template
 * on the scalar type so that forward-mode dual numbers give the exact
 * derivative of the discrete map (the reference gradient of the adjoint).
 *
 * Episode statistics per control step (the Task-1 error of Eq. (4), kinetic
 * energy, non-finite count) and the circle-tracking loss are computed in FP64.
 *
 * The Gym-style tasks of Sec. III (station keeping, circle, helix and
 * lemniscate tracking): the reference trajectories, the observation of
 * Eq. (2) (pose errors against the next m reference points, then nu), the
 * position error of Eq. (4) and the episode bookkeeping (counter, termination,
 * truncation, automatic reset) are written out step by step in FP64; their
 * readings are listed with the design notes.
 *
 * The split scheme of Sec. II is also written out: a physics engine steps the
 * rigid body (M_RB, C_RB, g_RB) by semi-implicit Euler while the hydrodynamic
 * wrench -M_A a_prev - C_A nu - D nu - g_A, computed from the current state
 * and the previous sub-step's acceleration a_prev, acts as an external force.
 */
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <omp.h>

namespace {

constexpr double kG0 = 9.81;
constexpr int kMaxThr = 8;
constexpr int kMaxState = 13 + kMaxThr;
constexpr int kNumTheta = 19;   // M_A(6), D_L(6), D_Q(6), B

/* ---- scalar types ------------------------------------------------------ */

struct Dual {
  double v, d;
  Dual(double x = 0.0) : v(x), d(0.0) {}
  Dual(double x, double dx) : v(x), d(dx) {}
};
inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
inline Dual operator/(Dual a, Dual b) {
  return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)};
}
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
inline Dual sqrt(Dual a) { double s = std::sqrt(a.v); return {s, a.d / (2.0 * s)}; }
inline Dual fabs(Dual a) { return a.v < 0.0 ? -a : a; }

inline double val(double x) { return x; }
inline double val(const Dual& x) { return x.v; }
inline double tan_of(double) { return 0.0; }
inline double tan_of(const Dual& x) { return x.d; }
inline void set_tan(double&, double) {}
inline void set_tan(Dual& x, double d) { x.d = d; }
using std::fabs;
using std::sqrt;

/* ---- vehicle description ---------------------------------------------- */

}  // namespace

extern "C" {
/* Raw preset numbers (SI).  Mirrored field-for-field by the ctypes shim. */
struct OrVehicle {
  double mass, inertia[3], r_g[3], r_b[3], added_mass[6], d_lin[6], d_quad[6], buoyancy;
  double thr_pos[kMaxThr][3], thr_dir[kMaxThr][3], f_max, thr_tau;
  int32_t n_thr, thr_map;
};
/* Task description (Sec. III).  Mirrored field-for-field by the ctypes shim.
 *   task           0 station keeping, 1 circle, 2 helix, 3 lemniscate
 *   lookahead      m reference points in the observation (tracking tasks)
 *   radius, omega  curve size (m) and rate of its parameter (rad/s)
 *   climb_rate     helix vertical rate (m/s along NED z)
 *   lookahead_dt   time between the look-ahead points (s)
 *   episode_steps  control steps per episode (truncation)
 *   max_error      position error (m) above which an episode terminates; 0: never */
struct OrTask {
  int32_t task, lookahead;
  double radius, omega, climb_rate, lookahead_dt;
  int32_t episode_steps, pad;
  double max_error;
};
}

namespace {

template <class T>
struct Body {
  T m, Ig[3], MA[6], DL[6], DQ[6], B;  // per-env (randomised) physical parameters
  double rg[3], rb[3];
  int n_thr, thr_map;
  double f_max, thr_tau;
  double Balloc[6][kMaxThr];
  bool lag() const { return thr_tau > 0.0; }
  int state_dim() const { return 13 + (lag() ? n_thr : 0); }
};

/* Thruster allocation: column i maps thrust f_i to the body wrench
 * [d_i ; r_i x d_i] (force along the unit direction, moment about the CO). */
void build_alloc(const OrVehicle& v, double B[6][kMaxThr]) {
  for (int r = 0; r < 6; ++r)
    for (int i = 0; i < kMaxThr; ++i) B[r][i] = 0.0;
  for (int i = 0; i < v.n_thr; ++i) {
    const double* r = v.thr_pos[i];
    const double* d = v.thr_dir[i];
    B[0][i] = d[0];
    B[1][i] = d[1];
    B[2][i] = d[2];
    B[3][i] = r[1] * d[2] - r[2] * d[1];
    B[4][i] = r[2] * d[0] - r[0] * d[2];
    B[5][i] = r[0] * d[1] - r[1] * d[0];
  }
}

/* Per-env body: nominal preset value times its multiplier (23 of them, order
 * m, I_g(3), M_A(6), D_L(6), D_Q(6), B).  dtheta, if given, seeds the tangent
 * of the 19 hydrodynamic parameters M_A, D_L, D_Q, B (absolute units). */
template <class T>
Body<T> make_body(const OrVehicle& v, const double* mult, const double* dtheta) {
  Body<T> b;
  auto mu = [&](int k) { return mult ? mult[k] : 1.0; };
  b.m = T(v.mass * mu(0));
  for (int i = 0; i < 3; ++i) b.Ig[i] = T(v.inertia[i] * mu(1 + i));
  for (int i = 0; i < 6; ++i) {
    b.MA[i] = T(v.added_mass[i] * mu(4 + i));
    b.DL[i] = T(v.d_lin[i] * mu(10 + i));
    b.DQ[i] = T(v.d_quad[i] * mu(16 + i));
  }
  b.B = T(v.buoyancy * mu(22));
  if (dtheta) {
    for (int i = 0; i < 6; ++i) {
      set_tan(b.MA[i], dtheta[i]);
      set_tan(b.DL[i], dtheta[6 + i]);
      set_tan(b.DQ[i], dtheta[12 + i]);
    }
    set_tan(b.B, dtheta[18]);
  }
  for (int i = 0; i < 3; ++i) {
    b.rg[i] = v.r_g[i];
    b.rb[i] = v.r_b[i];
  }
  b.n_thr = v.n_thr;
  b.thr_map = v.thr_map;
  b.f_max = v.f_max;
  b.thr_tau = v.thr_tau;
  build_alloc(v, b.Balloc);
  return b;
}

/* ---- small dense algebra ---------------------------------------------- */

/* S(a): the cross-product matrix, S(a) b = a x b. */
template <class T>
void skew(const T a[3], T S[3][3]) {
  S[0][0] = T(0.0); S[0][1] = -a[2];   S[0][2] = a[1];
  S[1][0] = a[2];   S[1][1] = T(0.0);  S[1][2] = -a[0];
  S[2][0] = -a[1];  S[2][1] = a[0];    S[2][2] = T(0.0);
}

template <class T>
void cross(const T a[3], const T b[3], T c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

/* Solve A x = b for symmetric positive definite 6x6 A by Cholesky (A = L L^T).
 * Returns false (and leaves NaN in x) if A is not positive definite. */
template <class T>
bool chol_solve6(const T A[6][6], const T b[6], T x[6]) {
  T L[6][6];
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) L[i][j] = T(0.0);
  for (int j = 0; j < 6; ++j) {
    T s = A[j][j];
    for (int k = 0; k < j; ++k) s -= L[j][k] * L[j][k];
    if (!(val(s) > 0.0)) {
      for (int i = 0; i < 6; ++i) x[i] = T(NAN);
      return false;
    }
    L[j][j] = sqrt(s);
    for (int i = j + 1; i < 6; ++i) {
      T t = A[i][j];
      for (int k = 0; k < j; ++k) t -= L[i][k] * L[j][k];
      L[i][j] = t / L[j][j];
    }
  }
  T y[6];
  for (int i = 0; i < 6; ++i) {
    T t = b[i];
    for (int k = 0; k < i; ++k) t -= L[i][k] * y[k];
    y[i] = t / L[i][i];
  }
  for (int i = 5; i >= 0; --i) {
    T t = y[i];
    for (int k = i + 1; k < 6; ++k) t -= L[k][i] * x[k];
    x[i] = t / L[i][i];
  }
  return true;
}

/* ---- the terms of Eq. (1) --------------------------------------------- */

/* M = M_RB + M_A.  M_RB about the CO with the CG at r_g:
 * [[m I3, -m S(r_g)], [m S(r_g), I_g - m S(r_g)^2]] (parallel-axis theorem). */
template <class T>
void mass_matrix(const Body<T>& b, T M[6][6]) {
  T rg[3] = {T(b.rg[0]), T(b.rg[1]), T(b.rg[2])};
  T S[3][3];
  skew(rg, S);
  T S2[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      T s = T(0.0);
      for (int k = 0; k < 3; ++k) s += S[i][k] * S[k][j];
      S2[i][j] = s;
    }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      M[i][j] = (i == j) ? b.m : T(0.0);
      M[i][3 + j] = -(b.m * S[i][j]);
      M[3 + i][j] = b.m * S[i][j];
      M[3 + i][3 + j] = ((i == j) ? b.Ig[i] : T(0.0)) - b.m * S2[i][j];
    }
  for (int i = 0; i < 6; ++i) M[i][i] += b.MA[i];
}

/* C(nu) built from the blocks of M (covers C_RB + C_A of Eq. (1)):
 * [[0, -S(M11 v + M12 w)], [-S(M11 v + M12 w), -S(M21 v + M22 w)]]. */
template <class T>
void coriolis_matrix(const T M[6][6], const T nu[6], T C[6][6]) {
  T a[3], bb[3];
  for (int i = 0; i < 3; ++i) {
    T s = T(0.0), t = T(0.0);
    for (int j = 0; j < 6; ++j) {
      s += M[i][j] * nu[j];
      t += M[3 + i][j] * nu[j];
    }
    a[i] = s;
    bb[i] = t;
  }
  T Sa[3][3], Sb[3][3];
  skew(a, Sa);
  skew(bb, Sb);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      C[i][j] = T(0.0);
      C[i][3 + j] = -Sa[i][j];
      C[3 + i][j] = -Sa[i][j];
      C[3 + i][3 + j] = -Sb[i][j];
    }
}

/* Body-to-NED rotation of a quaternion (w,x,y,z) by the unit-quaternion
 * formula, applied to the quaternion as given (RK4 stage values are not
 * normalised). */
template <class T>
void rotation(const T* q, T R[3][3]) {
  const T w = q[0], x = q[1], y = q[2], z = q[3];
  R[0][0] = T(1.0) - T(2.0) * (y * y + z * z);
  R[0][1] = T(2.0) * (x * y - w * z);
  R[0][2] = T(2.0) * (x * z + w * y);
  R[1][0] = T(2.0) * (x * y + w * z);
  R[1][1] = T(1.0) - T(2.0) * (x * x + z * z);
  R[1][2] = T(2.0) * (y * z - w * x);
  R[2][0] = T(2.0) * (x * z - w * y);
  R[2][1] = T(2.0) * (y * z + w * x);
  R[2][2] = T(1.0) - T(2.0) * (x * x + y * y);
}

/* Hamilton product a (x) b, scalar first. */
template <class T>
void quat_mul(const T* a, const T* b, T* c) {
  c[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
  c[1] = a[0] * b[1] + b[0] * a[1] + a[2] * b[3] - a[3] * b[2];
  c[2] = a[0] * b[2] + b[0] * a[2] + a[3] * b[1] - a[1] * b[3];
  c[3] = a[0] * b[3] + b[0] * a[3] + a[1] * b[2] - a[2] * b[1];
}

/* g_RB + g_A: weight W = m g0 at the CG, buoyancy B at the CB, expressed in
 * the body frame through k = R^T e_3 (the NED down axis seen from the body). */
template <class T>
void restoring(const Body<T>& b, const T R[3][3], T g[6]) {
  T k[3] = {R[2][0], R[2][1], R[2][2]};
  T W = b.m * T(kG0);
  T h[3];
  for (int i = 0; i < 3; ++i) h[i] = W * T(b.rg[i]) - b.B * T(b.rb[i]);
  T hk[3];
  cross(h, k, hk);
  for (int i = 0; i < 3; ++i) {
    g[i] = -((W - b.B) * k[i]);
    g[3 + i] = -hk[i];
  }
}

/* Throttle (Eq. (3)) -> commanded thrust: clamp to [-1,1], then F_max a or F_max a|a|. */
template <class T>
void thruster_command(const Body<T>& b, const T* a, T* fcmd) {
  for (int i = 0; i < b.n_thr; ++i) {
    T ai = a[i];
    if (val(ai) > 1.0) ai = T(1.0);
    if (val(ai) < -1.0) ai = T(-1.0);
    fcmd[i] = (b.thr_map == 1) ? T(b.f_max) * ai * fabs(ai) : T(b.f_max) * ai;
  }
}

/* Right-hand side x' = f(x) of the state x = [p(3), q(4), nu(6), f(n_thr if lag)]. */
template <class T>
void rhs(const Body<T>& b, const T* x, const T* fcmd, T* xd) {
  const T* q = x + 3;
  const T* nu = x + 7;
  const T* f = x + 13;
  T R[3][3];
  rotation(q, R);
  // kinematics: p' = R(q) v, q' = 1/2 q (x) (0, omega)
  for (int i = 0; i < 3; ++i) xd[i] = R[i][0] * nu[0] + R[i][1] * nu[1] + R[i][2] * nu[2];
  T om[4] = {T(0.0), nu[3], nu[4], nu[5]};
  T qd[4];
  quat_mul(q, om, qd);
  for (int i = 0; i < 4; ++i) xd[3 + i] = T(0.5) * qd[i];
  // control forces: tau = B_alloc * thrust
  const T* thrust = b.lag() ? f : fcmd;
  T tau[6];
  for (int r = 0; r < 6; ++r) {
    T s = T(0.0);
    for (int i = 0; i < b.n_thr; ++i) s += T(b.Balloc[r][i]) * thrust[i];
    tau[r] = s;
  }
  // Eq. (1) solved for nu'
  T M[6][6], C[6][6], g[6], r6[6], nud[6];
  mass_matrix(b, M);
  coriolis_matrix(M, nu, C);
  restoring(b, R, g);
  for (int i = 0; i < 6; ++i) {
    T Cnu = T(0.0);
    for (int j = 0; j < 6; ++j) Cnu += C[i][j] * nu[j];
    T Dnu = (b.DL[i] + b.DQ[i] * fabs(nu[i])) * nu[i];
    r6[i] = tau[i] - Cnu - Dnu - g[i];
  }
  chol_solve6(M, r6, nud);
  for (int i = 0; i < 6; ++i) xd[7 + i] = nud[i];
  if (b.lag())
    for (int i = 0; i < b.n_thr; ++i) xd[13 + i] = (fcmd[i] - f[i]) / T(b.thr_tau);
}

/* One classical RK4 substep (c = 0, 1/2, 1/2, 1; b = 1/6, 1/3, 1/3, 1/6) of
 * length dt with the command held, then q <- q / |q|. */
template <class T>
void rk4_substep(const Body<T>& b, T* x, const T* fcmd, double dt) {
  const int D = b.state_dim();
  T k1[kMaxState], k2[kMaxState], k3[kMaxState], k4[kMaxState], X[kMaxState];
  rhs(b, x, fcmd, k1);
  for (int i = 0; i < D; ++i) X[i] = x[i] + T(0.5 * dt) * k1[i];
  rhs(b, X, fcmd, k2);
  for (int i = 0; i < D; ++i) X[i] = x[i] + T(0.5 * dt) * k2[i];
  rhs(b, X, fcmd, k3);
  for (int i = 0; i < D; ++i) X[i] = x[i] + T(dt) * k3[i];
  rhs(b, X, fcmd, k4);
  for (int i = 0; i < D; ++i)
    x[i] = x[i] + T(dt / 6.0) * (k1[i] + T(2.0) * k2[i] + T(2.0) * k3[i] + k4[i]);
  T n = sqrt(x[3] * x[3] + x[4] * x[4] + x[5] * x[5] + x[6] * x[6]);
  for (int i = 3; i < 7; ++i) x[i] = x[i] / n;
}

/* One control step: the throttle frame a (n_thr values) is held for S substeps. */
template <class T>
void control_step(const Body<T>& b, T* x, const T* a, int S, double dt) {
  T fcmd[kMaxThr];
  thruster_command(b, a, fcmd);
  for (int s = 0; s < S; ++s) rk4_substep(b, x, fcmd, dt);
}

/* One sub-step of the split scheme (Sec. II): the hydrodynamic wrench of the
 * current state, with the added-mass term taken from the previous sub-step's
 * acceleration acc (6), acts on the rigid body as an external force; the
 * rigid body advances by semi-implicit Euler (velocity first, then position
 * with the new velocity and the old attitude, attitude with the new angular
 * rate), q <- q/|q|, the thruster lag by explicit Euler; acc <- the rigid
 * body's acceleration of this sub-step. */
template <class T>
void split_substep(const Body<T>& b, T* x, T* acc, const T* fcmd, double dt) {
  const T* q = x + 3;
  const T* nu = x + 7;
  T* f = x + 13;
  T R[3][3];
  rotation(q, R);
  const T* thrust = b.lag() ? f : fcmd;
  T tau[6];
  for (int r = 0; r < 6; ++r) {
    T s = T(0.0);
    for (int i = 0; i < b.n_thr; ++i) s += T(b.Balloc[r][i]) * thrust[i];
    tau[r] = s;
  }
  // rigid-body and added-mass matrices apart
  Body<T> rb = b;
  for (int i = 0; i < 6; ++i) rb.MA[i] = T(0.0);
  T MRB[6][6], MAd[6][6], CRB[6][6], CA[6][6];
  mass_matrix(rb, MRB);
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) MAd[i][j] = (i == j) ? b.MA[i] : T(0.0);
  coriolis_matrix(MRB, nu, CRB);
  coriolis_matrix(MAd, nu, CA);
  // restoring split: g_RB = -[W k ; W r_g x k] (gravity), g_A = [B k ; B r_b x k] (buoyancy)
  const T W = b.m * T(kG0);
  T k[3] = {R[2][0], R[2][1], R[2][2]};
  T gRB[6], gA[6];
  for (int i = 0; i < 3; ++i) {
    gRB[i] = -(W * k[i]);
    gA[i] = b.B * k[i];
  }
  T rgk[3], rbk[3];
  const T rg[3] = {T(b.rg[0]), T(b.rg[1]), T(b.rg[2])};
  const T rbv[3] = {T(b.rb[0]), T(b.rb[1]), T(b.rb[2])};
  cross(rg, k, rgk);
  cross(rbv, k, rbk);
  for (int i = 0; i < 3; ++i) {
    gRB[3 + i] = -(W * rgk[i]);
    gA[3 + i] = b.B * rbk[i];
  }
  T rhs6[6];
  for (int i = 0; i < 6; ++i) {
    T CRBnu = T(0.0), CAnu = T(0.0);
    for (int j = 0; j < 6; ++j) {
      CRBnu += CRB[i][j] * nu[j];
      CAnu += CA[i][j] * nu[j];
    }
    const T Dnu = (b.DL[i] + b.DQ[i] * fabs(nu[i])) * nu[i];
    const T tau_h = -(b.MA[i] * acc[i]) - CAnu - Dnu - gA[i];
    rhs6[i] = tau[i] + tau_h - CRBnu - gRB[i];
  }
  T a[6];
  chol_solve6(MRB, rhs6, a);
  T nun[6];
  for (int i = 0; i < 6; ++i) nun[i] = nu[i] + T(dt) * a[i];
  for (int i = 0; i < 3; ++i)
    x[i] = x[i] + T(dt) * (R[i][0] * nun[0] + R[i][1] * nun[1] + R[i][2] * nun[2]);
  T om[4] = {T(0.0), nun[3], nun[4], nun[5]};
  T qd[4];
  quat_mul(q, om, qd);
  T qn[4];
  for (int i = 0; i < 4; ++i) qn[i] = x[3 + i] + T(0.5 * dt) * qd[i];
  const T n = sqrt(qn[0] * qn[0] + qn[1] * qn[1] + qn[2] * qn[2] + qn[3] * qn[3]);
  for (int i = 0; i < 4; ++i) x[3 + i] = qn[i] / n;
  for (int i = 0; i < 6; ++i) {
    x[7 + i] = nun[i];
    acc[i] = a[i];
  }
  if (b.lag())
    for (int i = 0; i < b.n_thr; ++i) f[i] = f[i] + T(dt) * (fcmd[i] - f[i]) / T(b.thr_tau);
}

/* Kinetic energy 1/2 nu^T M nu. */
template <class T>
T kinetic_energy(const Body<T>& b, const T* nu) {
  T M[6][6];
  mass_matrix(b, M);
  T e = T(0.0);
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) e += nu[i] * M[i][j] * nu[j];
  return T(0.5) * e;
}

/* Circle-tracking loss of one control step: |p - p*|^2 + lam (1 - <q, q*>^2). */
template <class T>
T tracking_loss(const T* x, const double* pr, const double* qr, double lam) {
  T e = T(0.0);
  for (int i = 0; i < 3; ++i) {
    T d = x[i] - T(pr[i]);
    e += d * d;
  }
  T dot = T(0.0);
  for (int i = 0; i < 4; ++i) dot += x[3 + i] * T(qr[i]);
  return e + T(lam) * (T(1.0) - dot * dot);
}

int resolve_threads(int nthreads) { return nthreads > 0 ? nthreads : omp_get_max_threads(); }

/* ---- tasks of Sec. III ------------------------------------------------------- */

constexpr double kPi = 3.14159265358979323846;

/* Reference point p_r and reference heading psi_r at time t (s since the
 * episode began) of one env: centre c, curve phase ph, station-keeping yaw.
 * The curve parameter is s = omega t + ph; the reference heading of a
 * tracking task is the direction of the reference velocity dp_r/dt in the
 * horizontal plane, written out by the chain rule. */
void task_reference(const OrTask& tk, const double* c, double ph, double yaw, double t,
                    double* pr, double* psi) {
  const double R = tk.radius, w = tk.omega, s = w * t + ph;
  double off[3] = {0.0, 0.0, 0.0}, vel[3] = {0.0, 0.0, 0.0};
  switch (tk.task) {
    case 0:  // station keeping: a fixed point and heading
      for (int i = 0; i < 3; ++i) pr[i] = c[i];
      *psi = yaw;
      return;
    case 1:  // circle in the horizontal plane
    case 2:  // helix: the circle plus a constant vertical rate
      off[0] = R * std::cos(s);
      off[1] = R * std::sin(s);
      vel[0] = -R * w * std::sin(s);
      vel[1] = R * w * std::cos(s);
      if (tk.task == 2) {
        off[2] = tk.climb_rate * t;
        vel[2] = tk.climb_rate;
      }
      break;
    default: {  // lemniscate of Bernoulli, (x^2 + y^2)^2 = R^2 (x^2 - y^2)
      const double sn = std::sin(s), cs = std::cos(s), den = 1.0 + sn * sn;
      off[0] = R * cs / den;
      off[1] = R * sn * cs / den;
      // quotient rule on cos s / (1 + sin^2 s) and sin s cos s / (1 + sin^2 s)
      const double dxds = R * (-sn * den - cs * 2.0 * sn * cs) / (den * den);
      const double dyds = R * ((cs * cs - sn * sn) * den - sn * cs * 2.0 * sn * cs) / (den * den);
      vel[0] = w * dxds;
      vel[1] = w * dyds;
      break;
    }
  }
  for (int i = 0; i < 3; ++i) pr[i] = c[i] + off[i];
  *psi = std::atan2(vel[1], vel[0]);
}

/* Roll, pitch, yaw of the ZYX convention, R(q) = Rz(psi) Ry(theta) Rx(phi),
 * read off the rotation matrix. */
void euler_zyx(const double* q, double* rpy) {
  double R[3][3];
  rotation(q, R);
  const double s = std::max(-1.0, std::min(1.0, -R[2][0]));
  rpy[0] = std::atan2(R[2][1], R[2][2]);
  rpy[1] = std::asin(s);
  rpy[2] = std::atan2(R[1][0], R[0][0]);
}

/* Angle wrapped into (-pi, pi]. */
double wrap_angle(double a) {
  double r = std::remainder(a, 2.0 * kPi);
  if (r <= -kPi) r += 2.0 * kPi;
  return r;
}

int task_obs_dim(const OrTask& tk) { return tk.task == 0 ? 12 : 6 * tk.lookahead + 6; }

/* Observation of Eq. (2) at episode time t: the pose error against the
 * target (station keeping) or against each of the next m reference points at
 * t + i dl, i = 1..m (tracking), the reference attitude being level and
 * headed along the reference heading; then nu. */
void task_observe(const OrTask& tk, const double* x, const double* c, double ph, double yaw,
                  double t, double dl, double* obs) {
  double rpy[3];
  euler_zyx(x + 3, rpy);
  const int m = tk.task == 0 ? 1 : tk.lookahead;
  for (int i = 0; i < m; ++i) {
    const double ti = tk.task == 0 ? t : t + (i + 1) * dl;
    double pr[3], psi;
    task_reference(tk, c, ph, yaw, ti, pr, &psi);
    for (int k = 0; k < 3; ++k) obs[6 * i + k] = x[k] - pr[k];
    obs[6 * i + 3] = wrap_angle(rpy[0]);
    obs[6 * i + 4] = wrap_angle(rpy[1]);
    obs[6 * i + 5] = wrap_angle(rpy[2] - psi);
  }
  for (int k = 0; k < 6; ++k) obs[6 * m + k] = x[7 + k];
}

/* Position error of Eq. (4) at episode time t: |p - p_r(t)|. */
double task_error(const OrTask& tk, const double* x, const double* c, double ph, double yaw,
                  double t) {
  double pr[3], psi;
  task_reference(tk, c, ph, yaw, t, pr, &psi);
  double d2 = 0.0;
  for (int k = 0; k < 3; ++k) d2 += (x[k] - pr[k]) * (x[k] - pr[k]);
  return std::sqrt(d2);
}

}  // namespace


/* ======================================================================== */
/* C entry points (ctypes).  All arrays are FP64, row-major, SoA [comp][env]. */
/* ======================================================================== */
extern "C" {

int or_version() { return 1; }

int or_max_threads() { return omp_get_max_threads(); }

/* B_alloc, 6 x 8 row-major (columns beyond n_thr are zero). */
int or_alloc(const OrVehicle* v, double* out) {
  double B[6][kMaxThr];
  build_alloc(*v, B);
  std::memcpy(out, B, sizeof(B));
  return 0;
}

/* M = M_RB + M_A, 6 x 6 row-major; mult (23) may be NULL (nominal). */
int or_mass_matrix(const OrVehicle* v, const double* mult, double* out) {
  Body<double> b = make_body<double>(*v, mult, nullptr);
  double M[6][6];
  mass_matrix(b, M);
  std::memcpy(out, M, sizeof(M));
  return 0;
}

int or_coriolis_matrix(const double* M36, const double* nu, double* out) {
  double M[6][6], C[6][6];
  std::memcpy(M, M36, sizeof(M));
  coriolis_matrix(M, nu, C);
  std::memcpy(out, C, sizeof(C));
  return 0;
}

int or_restoring(const OrVehicle* v, const double* mult, const double* q, double* out) {
  Body<double> b = make_body<double>(*v, mult, nullptr);
  double R[3][3];
  rotation(q, R);
  restoring(b, R, out);
  return 0;
}

int or_rotation(const double* q, double* out) {
  double R[3][3];
  rotation(q, R);
  std::memcpy(out, R, sizeof(R));
  return 0;
}

/* x' for one env; x has 13 (+ n_thr with lag) entries, a has n_thr throttles. */
int or_rhs(const OrVehicle* v, const double* mult, const double* x, const double* a,
           double* xd) {
  Body<double> b = make_body<double>(*v, mult, nullptr);
  double fcmd[kMaxThr];
  thruster_command(b, a, fcmd);
  rhs(b, x, fcmd, xd);
  return 0;
}

/* Batched rollout.
 *   classes[n_classes], env_class[E] (NULL = all class 0)
 *   mult   [23][E]       or NULL (nominal)
 *   x0     [D][E]        D = io state width (13 + max lag thrusters); rows a class
 *                         does not use are ignored on input and written as 0
 *   act    [T][nmax][E]  throttles
 *   target [3][E]        or NULL (origin): station-keeping target for the stats
 *   traj   [T][D][E]     or NULL: state after each control step
 *   xT     [D][E]        final state (may be NULL)
 *   stats  [T][4]        or NULL: sum dist, max dist, sum KE over finite envs,
 *                         count of envs with a non-finite state
 * Returns 0, or -1 on a bad argument. */
int or_rollout(const OrVehicle* classes, int n_classes, const int32_t* env_class, int64_t E,
               const double* mult, const double* x0, int D, const double* act, int nmax,
               const double* target, int T, int S, double dt, double* traj, double* xT,
               double* stats, int nthreads) {
  if (E < 0 || T < 0 || S < 1 || n_classes < 1 || D < 13 || D > kMaxState) return -1;
  for (int c = 0; c < n_classes; ++c) {
    const OrVehicle& v = classes[c];
    if (v.n_thr < 1 || v.n_thr > nmax || v.n_thr > kMaxThr) return -1;
    if (v.thr_tau > 0.0 && 13 + v.n_thr > D) return -1;
  }
  std::vector<double> dist, ke;
  std::vector<unsigned char> bad;
  if (stats) {
    dist.assign((size_t)T * E, 0.0);
    ke.assign((size_t)T * E, 0.0);
    bad.assign((size_t)T * E, 0);
  }
#pragma omp parallel for schedule(dynamic, 16) num_threads(resolve_threads(nthreads))
  for (int64_t e = 0; e < E; ++e) {
    const int cls = env_class ? env_class[e] : 0;
    double m23[23];
    if (mult)
      for (int k = 0; k < 23; ++k) m23[k] = mult[(size_t)k * E + e];
    Body<double> b = make_body<double>(classes[cls], mult ? m23 : nullptr, nullptr);
    const int Dc = b.state_dim();
    double x[kMaxState];
    for (int i = 0; i < Dc; ++i) x[i] = x0[(size_t)i * E + e];
    for (int t = 0; t < T; ++t) {
      double a[kMaxThr];
      for (int i = 0; i < b.n_thr; ++i) a[i] = act[((size_t)t * nmax + i) * E + e];
      control_step(b, x, a, S, dt);
      if (traj)
        for (int i = 0; i < D; ++i) traj[((size_t)t * D + i) * E + e] = i < Dc ? x[i] : 0.0;
      if (stats) {
        bool finite = true;
        for (int i = 0; i < Dc; ++i) finite = finite && std::isfinite(x[i]);
        const size_t o = (size_t)t * E + e;
        bad[o] = !finite;
        if (finite) {
          double d2 = 0.0;
          for (int i = 0; i < 3; ++i) {
            double d = x[i] - (target ? target[(size_t)i * E + e] : 0.0);
            d2 += d * d;
          }
          dist[o] = std::sqrt(d2);
          ke[o] = kinetic_energy(b, x + 7);
        }
      }
    }
    if (xT)
      for (int i = 0; i < D; ++i) xT[(size_t)i * E + e] = i < Dc ? x[i] : 0.0;
  }
  if (stats) {
    for (int t = 0; t < T; ++t) {
      double sd = 0.0, md = 0.0, sk = 0.0, nb = 0.0;
      for (int64_t e = 0; e < E; ++e) {
        const size_t o = (size_t)t * E + e;
        if (bad[o]) {
          nb += 1.0;
          continue;
        }
        sd += dist[o];
        if (dist[o] > md) md = dist[o];
        sk += ke[o];
      }
      stats[4 * t + 0] = sd;
      stats[4 * t + 1] = md;
      stats[4 * t + 2] = sk;
      stats[4 * t + 3] = nb;
    }
  }
  return 0;
}

/* Kinetic energy 1/2 nu^T M nu of one env. */
double or_kinetic_energy(const OrVehicle* v, const double* mult, const double* nu) {
  Body<double> b = make_body<double>(*v, mult, nullptr);
  return kinetic_energy(b, nu);
}

/* Circle-tracking loss (one vehicle class, S substeps per control step):
 *   L_e = sum_{t=1..T} |p_t - p*_t|^2 + lam (1 - <q_t, q*_t>^2)
 * with x_t the state after control step t.  pref [T][3][E], qref [T][4][E].
 * loss[E] receives the per-env value. */
int or_track_loss(const OrVehicle* v, int64_t E, const double* mult, const double* x0, int D,
                  const double* act, int nmax, int T, int S, double dt, const double* pref,
                  const double* qref, double lam, double* loss, int nthreads) {
  if (v->n_thr > nmax || D < 13 || D > kMaxState) return -1;
#pragma omp parallel for schedule(dynamic, 4) num_threads(resolve_threads(nthreads))
  for (int64_t e = 0; e < E; ++e) {
    double m23[23];
    if (mult)
      for (int k = 0; k < 23; ++k) m23[k] = mult[(size_t)k * E + e];
    Body<double> b = make_body<double>(*v, mult ? m23 : nullptr, nullptr);
    double x[kMaxState];
    for (int i = 0; i < b.state_dim(); ++i) x[i] = x0[(size_t)i * E + e];
    double L = 0.0;
    for (int t = 0; t < T; ++t) {
      double a[kMaxThr];
      for (int i = 0; i < b.n_thr; ++i) a[i] = act[((size_t)t * nmax + i) * E + e];
      control_step(b, x, a, S, dt);
      double pr[3], qr[4];
      for (int i = 0; i < 3; ++i) pr[i] = pref[((size_t)t * 3 + i) * E + e];
      for (int i = 0; i < 4; ++i) qr[i] = qref[((size_t)t * 4 + i) * E + e];
      L += tracking_loss(x, pr, qr, lam);
    }
    loss[e] = L;
  }
  return 0;
}

/* Reference gradient of or_track_loss by forward-mode dual numbers: one dual
 * rollout per input direction, exact derivative of the discrete map.
 *   g_act   [T][nmax][E]  dL/d throttle (rows >= n_thr are 0; the clamp's
 *                         derivative is 0 outside [-1,1])
 *   g_theta [19][E]       dL/d (M_A(6), D_L(6), D_Q(6), B), absolute units
 *   g_x0    [D][E]        dL/d initial state (or NULL) */
int or_track_loss_grad(const OrVehicle* v, int64_t E, const double* mult, const double* x0,
                       int D, const double* act, int nmax, int T, int S, double dt,
                       const double* pref, const double* qref, double lam, double* loss,
                       double* g_act, double* g_theta, double* g_x0, int nthreads) {
  if (v->n_thr > nmax || D < 13 || D > kMaxState) return -1;
  const int Dc = 13 + (v->thr_tau > 0.0 ? v->n_thr : 0);
  const int n_act = T * v->n_thr;
  const int n_dir = n_act + kNumTheta + (g_x0 ? Dc : 0);
#pragma omp parallel for schedule(dynamic, 1) num_threads(resolve_threads(nthreads))
  for (int64_t e = 0; e < E; ++e) {
    double m23[23];
    if (mult)
      for (int k = 0; k < 23; ++k) m23[k] = mult[(size_t)k * E + e];
    std::vector<Dual> a((size_t)T * kMaxThr);
    for (int dir = 0; dir < n_dir; ++dir) {
      double dth[kNumTheta] = {0};
      int act_dir = -1, x_dir = -1;
      if (dir < n_act) act_dir = dir;
      else if (dir < n_act + kNumTheta) dth[dir - n_act] = 1.0;
      else x_dir = dir - n_act - kNumTheta;
      Body<Dual> b = make_body<Dual>(*v, mult ? m23 : nullptr, dth);
      Dual x[kMaxState];
      for (int i = 0; i < Dc; ++i) x[i] = Dual(x0[(size_t)i * E + e], i == x_dir ? 1.0 : 0.0);
      for (int t = 0; t < T; ++t)
        for (int i = 0; i < v->n_thr; ++i)
          a[(size_t)t * kMaxThr + i] =
              Dual(act[((size_t)t * nmax + i) * E + e], (t * v->n_thr + i) == act_dir ? 1.0 : 0.0);
      Dual L(0.0);
      for (int t = 0; t < T; ++t) {
        control_step(b, x, &a[(size_t)t * kMaxThr], S, dt);
        double pr[3], qr[4];
        for (int i = 0; i < 3; ++i) pr[i] = pref[((size_t)t * 3 + i) * E + e];
        for (int i = 0; i < 4; ++i) qr[i] = qref[((size_t)t * 4 + i) * E + e];
        L += tracking_loss(x, pr, qr, lam);
      }
      if (dir == 0 && loss) loss[e] = L.v;
      if (act_dir >= 0) {
        const int t = act_dir / v->n_thr, i = act_dir % v->n_thr;
        g_act[((size_t)t * nmax + i) * E + e] = L.d;
      } else if (x_dir < 0) {
        g_theta[(size_t)(dir - n_act) * E + e] = L.d;
      } else {
        g_x0[(size_t)x_dir * E + e] = L.d;
      }
    }
    for (int t = 0; t < T; ++t)
      for (int i = v->n_thr; i < nmax; ++i) g_act[((size_t)t * nmax + i) * E + e] = 0.0;
    if (g_x0)
      for (int i = Dc; i < D; ++i) g_x0[(size_t)i * E + e] = 0.0;
  }
  return 0;
}

/* Tangent (JVP) of one env's trajectory.  Inputs for the single env:
 *   mult[23] (or NULL), x0[Dc], act[T][nmax]; tangents dact[T][nmax] (or NULL),
 *   dtheta[19] (or NULL), dx0[Dc] (or NULL).
 * Outputs traj[T][Dc] and dtraj[T][Dc]. */
int or_jvp(const OrVehicle* v, const double* mult, const double* x0, const double* act,
           int nmax, int T, int S, double dt, const double* dact, const double* dtheta,
           const double* dx0, double* traj, double* dtraj) {
  if (v->n_thr > nmax) return -1;
  Body<Dual> b = make_body<Dual>(*v, mult, dtheta);
  const int Dc = b.state_dim();
  Dual x[kMaxState];
  for (int i = 0; i < Dc; ++i) x[i] = Dual(x0[i], dx0 ? dx0[i] : 0.0);
  for (int t = 0; t < T; ++t) {
    Dual a[kMaxThr];
    for (int i = 0; i < b.n_thr; ++i)
      a[i] = Dual(act[(size_t)t * nmax + i], dact ? dact[(size_t)t * nmax + i] : 0.0);
    control_step(b, x, a, S, dt);
    for (int i = 0; i < Dc; ++i) {
      traj[(size_t)t * Dc + i] = x[i].v;
      dtraj[(size_t)t * Dc + i] = x[i].d;
    }
  }
  return 0;
}

}  // extern "C"

/* ---- tasks of Sec. III (C entry points) ------------------------------------- */
extern "C" {

/* Reference point pr[3] and heading *psi of one env at episode time t. */
int or_task_reference(const OrTask* tk, const double* c, double phase, double yaw, double t,
                      double* pr, double* psi) {
  if (!tk || tk->task < 0 || tk->task > 3) return -1;
  task_reference(*tk, c, phase, yaw, t, pr, psi);
  return 0;
}

/* ZYX roll, pitch, yaw of the unit quaternion q (scalar first). */
int or_euler_zyx(const double* q, double* rpy) {
  euler_zyx(q, rpy);
  return 0;
}

/* Observation width of a task: 12 (station keeping) or 6 m + 6 (tracking). */
int or_task_obs_dim(const OrTask* tk) { return task_obs_dim(*tk); }

/* Observations [obs_dim][E] of the states x [D][E] at episode step k[E]
 * (time k * dt_ctrl); centre [3][E], phase [E], yaw [E] (or NULL: 0). */
int or_task_observe(const OrTask* tk, int64_t E, const double* x, int D, const double* center,
                    const double* phase, const double* yaw, const int32_t* k, double dt_ctrl,
                    double* obs) {
  if (!tk || tk->task < 0 || tk->task > 3 || (tk->task != 0 && tk->lookahead < 1)) return -1;
  if (D < 13 || D > kMaxState) return -1;
  const int od = task_obs_dim(*tk);
  const double dl = tk->lookahead_dt > 0.0 ? tk->lookahead_dt : dt_ctrl;
  for (int64_t e = 0; e < E; ++e) {
    double xe[kMaxState], c[3], o[6 * 16 + 6];
    for (int i = 0; i < D; ++i) xe[i] = x[(size_t)i * E + e];
    for (int i = 0; i < 3; ++i) c[i] = center[(size_t)i * E + e];
    task_observe(*tk, xe, c, phase[e], yaw ? yaw[e] : 0.0, (k ? k[e] : 0) * dt_ctrl, dl, o);
    for (int i = 0; i < od; ++i) obs[(size_t)i * E + e] = o[i];
  }
  return 0;
}

/* T Gym-style steps of every env: each step is one control step (S substeps
 * of dt with the throttle frame held), then the episode counter advances, the
 * position error of Eq. (4) is taken at the new time, and the episode ends
 * terminated (done 1: non-finite state, or error above max_error > 0) or
 * truncated (done 2: episode_steps reached).  An ended episode restarts at
 * once from the env's column of reset_state [D][E] (NULL: at rest at the
 * origin, identity attitude, no thrust), with the parameters nominal x
 * reset_mult [23][E] if given (else unchanged) and the counter at 0; the
 * observation after the step is that of the new episode.
 *   x0 [D][E], act [T][nmax][E], mult [23][E] or NULL, k0 [E] or NULL (0)
 *   obs [(T + 1)][obs_dim][E] (before the first step, then after each),
 *   err [T][E], done [T][E] (int32), xT [D][E], kT [E] (int32), each or NULL */
int or_task_rollout(const OrVehicle* classes, int n_classes, const int32_t* env_class, int64_t E,
                    const double* mult, const double* x0, int D, const double* act, int nmax,
                    int T, int S, double dt, const OrTask* tk, const double* center,
                    const double* phase, const double* yaw, const int32_t* k0,
                    const double* reset_state, const double* reset_mult, double* obs,
                    double* err, int32_t* done, double* xT, int32_t* kT, int nthreads) {
  if (E < 0 || T < 0 || S < 1 || n_classes < 1 || D < 13 || D > kMaxState || !tk) return -1;
  if (tk->task < 0 || tk->task > 3 || (tk->task != 0 && (tk->lookahead < 1 || tk->lookahead > 16)))
    return -1;
  if (tk->episode_steps < 1) return -1;
  for (int c = 0; c < n_classes; ++c) {
    const OrVehicle& v = classes[c];
    if (v.n_thr < 1 || v.n_thr > nmax || v.n_thr > kMaxThr) return -1;
    if (v.thr_tau > 0.0 && 13 + v.n_thr > D) return -1;
  }
  const int od = task_obs_dim(*tk);
  const double dtc = S * dt;
  const double dl = tk->lookahead_dt > 0.0 ? tk->lookahead_dt : dtc;
#pragma omp parallel for schedule(dynamic, 16) num_threads(resolve_threads(nthreads))
  for (int64_t e = 0; e < E; ++e) {
    const int cls = env_class ? env_class[e] : 0;
    double m23[23], c[3], o[6 * 16 + 6];
    if (mult)
      for (int k = 0; k < 23; ++k) m23[k] = mult[(size_t)k * E + e];
    Body<double> b = make_body<double>(classes[cls], mult ? m23 : nullptr, nullptr);
    const int Dc = b.state_dim();
    for (int i = 0; i < 3; ++i) c[i] = center[(size_t)i * E + e];
    const double ph = phase[e], yw = yaw ? yaw[e] : 0.0;
    double x[kMaxState];
    for (int i = 0; i < Dc; ++i) x[i] = x0[(size_t)i * E + e];
    int32_t k = k0 ? k0[e] : 0;
    auto put_obs = [&](int slot) {
      if (!obs) return;
      task_observe(*tk, x, c, ph, yw, k * dtc, dl, o);
      for (int i = 0; i < od; ++i) obs[((size_t)slot * od + i) * E + e] = o[i];
    };
    put_obs(0);
    for (int t = 0; t < T; ++t) {
      double a[kMaxThr];
      for (int i = 0; i < b.n_thr; ++i) a[i] = act[((size_t)t * nmax + i) * E + e];
      control_step(b, x, a, S, dt);
      k += 1;
      bool finite = true;
      for (int i = 0; i < Dc; ++i) finite = finite && std::isfinite(x[i]);
      const double ee = task_error(*tk, x, c, ph, yw, k * dtc);
      const bool term = !finite || (tk->max_error > 0.0 && !(ee <= tk->max_error));
      const int32_t d = term ? 1 : (k >= tk->episode_steps ? 2 : 0);
      if (err) err[(size_t)t * E + e] = ee;
      if (done) done[(size_t)t * E + e] = d;
      if (d) {
        for (int i = 0; i < Dc; ++i)
          x[i] = reset_state ? reset_state[(size_t)i * E + e] : (i == 3 ? 1.0 : 0.0);
        k = 0;
        if (reset_mult) {
          for (int j = 0; j < 23; ++j) m23[j] = reset_mult[(size_t)j * E + e];
          b = make_body<double>(classes[cls], m23, nullptr);
        }
      }
      put_obs(t + 1);
    }
    if (xT)
      for (int i = 0; i < D; ++i) xT[(size_t)i * E + e] = i < Dc ? x[i] : 0.0;
    if (kT) kT[e] = k;
  }
  return 0;
}

}  // extern "C"

/* ---- split scheme of Sec. II (C entry point) ---------------------------------- */
extern "C" {

/* T control steps of the split scheme for every env (S sub-steps of dt each,
 * the throttle frame held), from states x0 [D][E] and previous-sub-step
 * accelerations acc0 [6][E] (NULL: 0).  traj [T][D][E], xT [D][E] and accT
 * [6][E] as for or_rollout, each or NULL. */
int or_split_rollout(const OrVehicle* classes, int n_classes, const int32_t* env_class, int64_t E,
                     const double* mult, const double* x0, const double* acc0, int D,
                     const double* act, int nmax, int T, int S, double dt, double* traj,
                     double* xT, double* accT, int nthreads) {
  if (E < 0 || T < 0 || S < 1 || n_classes < 1 || D < 13 || D > kMaxState) return -1;
  for (int c = 0; c < n_classes; ++c) {
    const OrVehicle& v = classes[c];
    if (v.n_thr < 1 || v.n_thr > nmax || v.n_thr > kMaxThr) return -1;
    if (v.thr_tau > 0.0 && 13 + v.n_thr > D) return -1;
  }
#pragma omp parallel for schedule(dynamic, 16) num_threads(resolve_threads(nthreads))
  for (int64_t e = 0; e < E; ++e) {
    const int cls = env_class ? env_class[e] : 0;
    double m23[23];
    if (mult)
      for (int k = 0; k < 23; ++k) m23[k] = mult[(size_t)k * E + e];
    Body<double> b = make_body<double>(classes[cls], mult ? m23 : nullptr, nullptr);
    const int Dc = b.state_dim();
    double x[kMaxState], acc[6];
    for (int i = 0; i < Dc; ++i) x[i] = x0[(size_t)i * E + e];
    for (int i = 0; i < 6; ++i) acc[i] = acc0 ? acc0[(size_t)i * E + e] : 0.0;
    for (int t = 0; t < T; ++t) {
      double a[kMaxThr], fcmd[kMaxThr];
      for (int i = 0; i < b.n_thr; ++i) a[i] = act[((size_t)t * nmax + i) * E + e];
      thruster_command(b, a, fcmd);
      for (int s = 0; s < S; ++s) split_substep(b, x, acc, fcmd, dt);
      if (traj)
        for (int i = 0; i < D; ++i) traj[((size_t)t * D + i) * E + e] = i < Dc ? x[i] : 0.0;
    }
    if (xT)
      for (int i = 0; i < D; ++i) xT[(size_t)i * E + e] = i < Dc ? x[i] : 0.0;
    if (accT)
      for (int i = 0; i < 6; ++i) accT[(size_t)i * E + e] = acc[i];
  }
  return 0;
}

}  // extern "C"
