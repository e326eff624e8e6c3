// Host-side check of the kernels' reverse-mode code (fossen_adjoint.h) in FP64:
// every vector-Jacobian product is compared with central finite differences of
// the same forward functions (fossen_device.h) run in double precision.
// Runs on the CPU only (no kernel is launched).  Prints the worst relative
// error per quantity and exits non-zero if one exceeds the tolerance.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>

#include "fossen_adjoint.h"

using namespace mg;

namespace {

struct Theta {   // m, I(3), MA(6), DL(6), DQ(6), B
  double p[23];
};

// per-env constants of the structured mass matrix (diagonal I_g and M_A,
// r_g = (0,0,zg), r_b = (0,0,zb)), used here to perturb theta consistently
EnvConstT<double> make_env(const Theta& th, double zg, double zb) {
  const double* p = th.p;
  EnvConstT<double> P;
  const double m = p[0];
  P.Muu = m + p[4]; P.Mvv = m + p[5]; P.Mww = m + p[6];
  P.Mpp = p[1] + m * zg * zg + p[7]; P.Mqq = p[2] + m * zg * zg + p[8]; P.Mrr = p[3] + p[9];
  P.Muq = m * zg; P.Mvp = -m * zg;
  const double duq = P.Muu * P.Mqq - P.Muq * P.Muq, dvp = P.Mvv * P.Mpp - P.Mvp * P.Mvp;
  P.Iuu = P.Mqq / duq; P.Iqq = P.Muu / duq; P.Iuq = -P.Muq / duq;
  P.Ivv = P.Mpp / dvp; P.Ipp = P.Mvv / dvp; P.Ivp = -P.Mvp / dvp;
  P.Iww = 1.0 / P.Mww; P.Irr = 1.0 / P.Mrr;
  for (int i = 0; i < 6; ++i) {
    P.dl[i] = p[10 + i];
    P.dq[i] = p[16 + i];
  }
  const double W = m * 9.81, B = p[22];
  P.wmb = W - B;
  P.hz = W * zg - B * zb;
  return P;
}

template <int N>
ClassConst make_class(std::mt19937_64& g, bool lag, int map, double dt, int S) {
  std::uniform_real_distribution<double> U(-1, 1);
  ClassConst c;
  std::memset(&c, 0, sizeof c);
  for (int k = 0; k < 6; ++k)
    for (int i = 0; i < N; ++i) c.B[k][i] = (float)(k < 3 ? U(g) : 0.2 * U(g));
  c.f_max = 40.0f;
  const double tau = 0.05;
  c.inv_tau = lag ? (float)(1.0 / tau) : 0.0f;
  const double z = lag ? dt / tau : 0.0;
  c.sigma2 = (float)(1 - z / 2);
  c.sigma3 = (float)(1 - z / 2 + z * z / 4);
  c.sigma4 = (float)(1 - z + z * z / 2 - z * z * z / 4);
  c.rho = (float)(1 - z + z * z / 2 - z * z * z / 6 + z * z * z * z / 24);
  c.rho_s = (float)std::pow(1 - z + z * z / 2 - z * z * z / 6 + z * z * z * z / 24, (double)S);
  c.n_thr = N;
  c.thr_map = map;
  c.lag = lag;
  return c;
}

double worst = 0.0;
int failures = 0;

void report(const char* what, double got, double fd, double scale, double tol) {
  const double err = std::fabs(got - fd) / std::max(1e-8, scale);
  if (err > worst) worst = err;
  if (err > tol) {
    ++failures;
    std::printf("FAIL %-28s vjp % .10e  fd % .10e  rel %.2e\n", what, got, fd, err);
  }
}

// one control step: throttle -> f_cmd -> S sub-steps; returns <lam, x_out>
template <int N, bool LAG>
double control_step_dot(const ClassConst& cc, const EnvConstT<double>& P, const double* x0,
                        const double (&a)[N], int S, double dt, const double* lam) {
  constexpr int D = Dims<N, LAG>::D;
  double x[D], fcmd[N], gcmd[6];
  for (int i = 0; i < D; ++i) x[i] = x0[i];
  thrust_command<N>(cc, a, fcmd);
  command_wrench<N>(cc, fcmd, gcmd);
  const StepConstT<double> sc = make_step_const_host(cc, dt);
  control_step<N, LAG>(x, P, half_step_inverse(P, sc.h2), cc, fcmd, gcmd, sc, S, (double)cc.rho_s);
  double d = 0;
  for (int i = 0; i < D; ++i) d += lam[i] * x[i];
  return d;
}

template <int N, bool LAG>
void check_case(unsigned seed, int map, int S, double dt) {
  constexpr int D = Dims<N, LAG>::D;
  std::mt19937_64 g(seed);
  std::uniform_real_distribution<double> U(-1, 1);
  const ClassConst cc = make_class<N>(g, LAG, map, dt, S);
  Theta th;
  const double nominal[23] = {11.5, 0.16, 0.16, 0.16, 5.5, 12.7, 14.6, 0.12, 0.12, 0.12,
                              4, 6, 5, 0.07, 0.07, 0.07, 18, 21, 37, 0.45, 0.45, 0.45,
                              11.5 * 9.81 * 0.97};
  for (int i = 0; i < 23; ++i) th.p[i] = nominal[i] * (1 + 0.2 * U(g));
  const double zg = 0.02, zb = -0.01;
  const EnvConstT<double> P = make_env(th, zg, zb);
  double x0[D];
  for (int i = 0; i < D; ++i) x0[i] = U(g);
  double qn = 0;
  for (int i = 3; i < 7; ++i) qn += x0[i] * x0[i];
  for (int i = 3; i < 7; ++i) x0[i] /= std::sqrt(qn);
  for (int i = 7; i < 13; ++i) x0[i] *= 1.5;
  for (int i = 13; i < D; ++i) x0[i] *= 30.0;
  double a[N];
  for (int i = 0; i < N; ++i) a[i] = 0.9 * U(g);
  double lam_out[D];
  for (int i = 0; i < D; ++i) lam_out[i] = U(g);

  // reverse mode through one control step: store the sub-step inputs (with the
  // lag states of each sub-step, f_cmd + rho^s (f - f_cmd)), sweep back
  double xs[64][D], x[D], fcmd[N], gcmd[6], fs[N];
  for (int i = 0; i < D; ++i) x[i] = x0[i];
  thrust_command<N>(cc, a, fcmd);
  command_wrench<N>(cc, fcmd, gcmd);
  for (int i = 0; i < N; ++i) fs[i] = LAG ? x[13 + i] : 0.0;
  double dg[6];
  begin_control_step<N, LAG>(cc, x, fcmd, dg, (double)cc.rho_s);
  const StepConstT<double> sc = make_step_const_host(cc, dt);
  double m[6];
  momentum(P, x + 7, m);
  for (int s = 0; s < S; ++s) {
    for (int i = 0; i < 13; ++i) xs[s][i] = x[i];
    for (int i = 13; i < D; ++i) {
      xs[s][i] = fs[i - 13];
      fs[i - 13] = sc.rho * (fs[i - 13] - fcmd[i - 13]) + fcmd[i - 13];
    }
    rk4_substep<N, LAG>(x, m, P, half_step_inverse(P, sc.h2), gcmd, dg, sc);
  }
  double lam[D], fcb[N] = {0}, gcb[6] = {0}, ab[N];
  for (int i = 0; i < D; ++i) lam[i] = lam_out[i];
  ThetaBar<double> thb;
  theta_bar_zero(thb);
  for (int s = S - 1; s >= 0; --s)
    rk4_substep_vjp<N, LAG>(xs[s], P, cc, fcmd, gcmd, dt, lam, fcb, gcb, thb);
  throttle_vjp<N>(cc, a, fcb, gcb, ab);

  char name[64];
  const double tol = 2e-6;
  // state
  for (int j = 0; j < D; ++j) {
    const double h = 1e-6;
    double xp[D], xm[D];
    for (int i = 0; i < D; ++i) xp[i] = xm[i] = x0[i];
    xp[j] += h;
    xm[j] -= h;
    const double fd = (control_step_dot<N, LAG>(cc, P, xp, a, S, dt, lam_out) -
                       control_step_dot<N, LAG>(cc, P, xm, a, S, dt, lam_out)) / (2 * h);
    std::snprintf(name, sizeof name, "N%d lag%d map%d dx[%d]", N, (int)LAG, map, j);
    report(name, lam[j], fd, std::max(1.0, std::fabs(fd)), tol);
  }
  // throttles
  for (int j = 0; j < N; ++j) {
    const double h = 1e-6;
    double ap[N], am[N];
    for (int i = 0; i < N; ++i) ap[i] = am[i] = a[i];
    ap[j] += h;
    am[j] -= h;
    const double fd = (control_step_dot<N, LAG>(cc, P, x0, ap, S, dt, lam_out) -
                       control_step_dot<N, LAG>(cc, P, x0, am, S, dt, lam_out)) / (2 * h);
    std::snprintf(name, sizeof name, "N%d lag%d map%d da[%d]", N, (int)LAG, map, j);
    report(name, ab[j], fd, std::max(1.0, std::fabs(fd)), tol);
  }
  // theta = M_A, D_L, D_Q, B
  const double thbar[19] = {thb.ma[0], thb.ma[1], thb.ma[2], thb.ma[3], thb.ma[4], thb.ma[5],
                            thb.dl[0], thb.dl[1], thb.dl[2], thb.dl[3], thb.dl[4], thb.dl[5],
                            thb.dq[0], thb.dq[1], thb.dq[2], thb.dq[3], thb.dq[4], thb.dq[5],
                            -thb.wmb - zb * thb.hz};
  for (int j = 0; j < 19; ++j) {
    const double h = 1e-6 * std::max(1.0, std::fabs(th.p[4 + j]));
    Theta tp = th, tm = th;
    tp.p[4 + j] += h;
    tm.p[4 + j] -= h;
    const double fd = (control_step_dot<N, LAG>(cc, make_env(tp, zg, zb), x0, a, S, dt, lam_out) -
                       control_step_dot<N, LAG>(cc, make_env(tm, zg, zb), x0, a, S, dt, lam_out)) /
                      (2 * h);
    std::snprintf(name, sizeof name, "N%d lag%d map%d dtheta[%d]", N, (int)LAG, map, j);
    report(name, thbar[j], fd, std::max(1.0, std::fabs(fd)), tol);
  }
}

}  // namespace

int main() {
  for (unsigned seed = 1; seed <= 5; ++seed) {
    check_case<6, false>(seed, 0, 1, 0.01);      // BlueROV2, linear map, no lag
    check_case<8, true>(seed, 1, 4, 0.005);      // Heavy, quadratic map, lag, 4 sub-steps
    check_case<6, true>(seed, 1, 3, 0.005);      // BlueROV2 with lag
    check_case<1, false>(seed, 1, 2, 0.02);
  }
  std::printf("vjp check: worst relative error %.3e, %d failures\n", worst, failures);
  return failures ? 1 : 0;
}
