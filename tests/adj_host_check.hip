// CPU run of the FP32 adjoint backward's source (fossen_adjoint.h): the
// per-env backward adj_bwd_env, host and device code, is run on the host for
// every env of small rollouts, in four forms that must agree bitwise:
//   current   the backward that recomputes each segment with its own loop
//   factored  the same with that loop replaced by a call of recompute_segment
//             (the form that once gave wrong gradients on the GPU for the
//             one-wave 8-thruster lag kernel)
//   whole     every segment recomputed first by recompute_segment into a
//             whole-rollout buffer, then the sweep-only backward
//   prefetch  the sweep that loads each next sub-step's inputs one step ahead
// Built with AddressSanitizer and UndefinedBehaviorSanitizer for the host, so
// that an out-of-bounds access or undefined operation in that source is
// reported.  No kernel is launched.  Prints "N failures".
#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "fossen_adjoint.h"

using namespace mg;

namespace {

int failures = 0;

// the step factors as make_step_const forms them (without the register move)
StepConstT<float> step_const(const ClassConst& cc, float dt) {
  StepConstT<float> k;
  const float h2 = 0.5f * dt, h6 = dt * (1.0f / 6.0f);
  k.h2 = h2;
  k.h2q = 0.5f * h2;
  k.dt = dt;
  k.dtq = 0.5f * dt;
  k.h6 = h6;
  k.h6q = 0.5f * h6;
  k.two = 2.0f;
  k.third = 1.0f / 3.0f;
  k.s2 = cc.sigma2;
  k.s3 = cc.sigma3;
  k.s4 = cc.sigma4;
  k.rho = cc.rho;
  return k;
}

// the backward with the recomputation loop factored into recompute_segment
template <int N, bool LAG>
void adj_bwd_env_factored(const AdjArgs& a, const ClassConst& cc, const EnvConst& P,
                          const StepConstT<float>& sc, const HalfInvT<float>& A, int64_t j,
                          int64_t c) {
  constexpr int D = Dims<N, LAG>::D;
  const int K = a.ckpt_every, S = a.substeps;
  const int nseg = (a.T + K - 1) / K;
  float lam[D];
  for (int i = 0; i < D; ++i) lam[i] = 0.0f;
  ThetaBar<float> thb;
  theta_bar_zero(thb);
  for (int seg = nseg - 1; seg >= 0; --seg) {
    const int t0 = seg * K, t1 = std::min(a.T, t0 + K);
    float x[D];
    const float* ck = a.ckpt + (int64_t)seg * a.D * a.E + c;
    for (int i = 0; i < D; ++i) x[i] = ck[i * a.E];
    recompute_segment<N, LAG>(a, cc, P, A, sc, x, t0, t1, t0, j, c);
    for (int t = t1 - 1; t >= t0; --t) {
      const float* gt = a.gtraj + (int64_t)t * a.D * a.E + c;
      for (int i = 0; i < D; ++i) lam[i] += gt[i * a.E];
      float act[N], fcmd[N], gcmd[6], fcb[N], gcb[6], ab[N];
      load_command<N>(cc, a, t, c, act, fcmd, gcmd);
      for (int i = 0; i < N; ++i) fcb[i] = 0.0f;
      for (int k = 0; k < 6; ++k) gcb[k] = 0.0f;
      for (int s = S - 1; s >= 0; --s) {
        float y[D];
        const float* sb = a.segbuf + (int64_t)((t - t0) * S + s) * D * a.Ep + j;
        for (int i = 0; i < D; ++i) y[i] = sb[i * a.Ep];
        rk4_substep_vjp<N, LAG>(y, P, cc, fcmd, gcmd, a.dt, lam, fcb, gcb, thb);
      }
      throttle_vjp<N>(cc, act, fcb, gcb, ab);
      float* ga = a.gact + (int64_t)t * a.n_max * a.E + c;
      for (int i = 0; i < N; ++i) ga[i * a.E] = ab[i];
      for (int i = N; i < a.n_max; ++i) ga[i * a.E] = 0.0f;
    }
  }
  for (int i = 0; i < 6; ++i) {
    a.gtheta[i * a.E + c] = thb.ma[i];
    a.gtheta[(6 + i) * a.E + c] = thb.dl[i];
    a.gtheta[(12 + i) * a.E + c] = thb.dq[i];
  }
  a.gtheta[18 * a.E + c] = -thb.wmb - a.zb * thb.hz;
  if (a.gx0) {
    for (int i = 0; i < D; ++i) a.gx0[i * a.E + c] = lam[i];
    for (int i = D; i < a.D; ++i) a.gx0[i * a.E + c] = 0.0f;
  }
}

template <int N>
ClassConst make_class(std::mt19937_64& g, bool lag, int map, double dt, int S) {
  std::uniform_real_distribution<double> U(-1, 1);
  ClassConst c;
  std::memset(&c, 0, sizeof c);
  for (int k = 0; k < 6; ++k)
    for (int i = 0; i < N; ++i) c.B[k][i] = (float)(k < 3 ? U(g) : 0.2 * U(g));
  c.f_max = 40.0f;
  const double z = lag ? dt / 0.05 : 0.0;
  const double rho = 1 - z + z * z / 2 - z * z * z / 6 + z * z * z * z / 24;
  c.inv_tau = lag ? 20.0f : 0.0f;
  c.sigma2 = (float)(1 - z / 2);
  c.sigma3 = (float)(1 - z / 2 + z * z / 4);
  c.sigma4 = (float)(1 - z + z * z / 2 - z * z * z / 4);
  c.rho = (float)rho;
  c.rho_s = (float)std::pow(rho, (double)S);
  c.n_thr = N;
  c.thr_map = map;
  c.lag = lag;
  return c;
}

// per-env constants of a randomised BlueROV2-like mass matrix (diagonal
// inertia and added mass, z_g = 0.02), formed in double and rounded once
EnvConst make_env(std::mt19937_64& g) {
  std::uniform_real_distribution<double> U(0.8, 1.2);
  const double m = 11.5 * U(g), zg = 0.02, zb = 0.0;
  const double I[3] = {0.16 * U(g), 0.16 * U(g), 0.16 * U(g)};
  const double MA[6] = {5.5 * U(g), 12.7 * U(g), 14.6 * U(g), 0.12 * U(g), 0.12 * U(g),
                        0.12 * U(g)};
  const double Muu = m + MA[0], Mvv = m + MA[1], Mww = m + MA[2];
  const double Mpp = I[0] + m * zg * zg + MA[3], Mqq = I[1] + m * zg * zg + MA[4];
  const double Mrr = I[2] + MA[5], Muq = m * zg, Mvp = -m * zg;
  const double duq = Muu * Mqq - Muq * Muq, dvp = Mvv * Mpp - Mvp * Mvp;
  EnvConst P;
  P.Muu = (float)Muu; P.Mvv = (float)Mvv; P.Mww = (float)Mww;
  P.Mpp = (float)Mpp; P.Mqq = (float)Mqq; P.Mrr = (float)Mrr;
  P.Muq = (float)Muq; P.Mvp = (float)Mvp;
  P.Iuu = (float)(Mqq / duq); P.Iqq = (float)(Muu / duq); P.Iuq = (float)(-Muq / duq);
  P.Ivv = (float)(Mpp / dvp); P.Ipp = (float)(Mvv / dvp); P.Ivp = (float)(-Mvp / dvp);
  P.Iww = (float)(1.0 / Mww); P.Irr = (float)(1.0 / Mrr);
  const double DL[6] = {4, 6, 5, 0.07, 0.07, 0.07}, DQ[6] = {18, 21, 37, 0.45, 0.45, 0.45};
  for (int i = 0; i < 6; ++i) {
    P.dl[i] = (float)(DL[i] * U(g));
    P.dq[i] = (float)(DQ[i] * U(g));
  }
  const double W = m * 9.81, B = W * U(g);
  P.wmb = (float)(W - B);
  P.hz = (float)(W * zg - B * zb);
  return P;
}

template <int N, bool LAG>
void check(unsigned seed, int E, int T, int K, int S, int map, float dt) {
  constexpr int D = Dims<N, LAG>::D;
  const int Dio = D + 1;              // I/O width wider than the class's, as with mixed classes
  const int n_max = N + 1;            // and a wider throttle frame
  std::mt19937_64 g(seed);
  std::uniform_real_distribution<double> U(-1, 1);
  const ClassConst cc = make_class<N>(g, LAG, map, dt, S);
  const StepConstT<float> sc = step_const(cc, dt);
  std::vector<EnvConst> Ps;
  for (int e = 0; e < E; ++e) Ps.push_back(make_env(g));
  const int nseg = (T + K - 1) / K;
  // inputs: checkpoints from a forward over the segments, throttles, dL/d traj
  std::vector<float> act((size_t)T * n_max * E), gtraj((size_t)T * Dio * E),
      ckpt((size_t)nseg * Dio * E, 0.0f);
  for (auto& v : act) v = (float)(1.1 * U(g));
  for (auto& v : gtraj) v = (float)U(g);
  for (int e = 0; e < E; ++e) {
    float x[D];
    for (int i = 0; i < D; ++i) x[i] = (float)(i < 13 ? 0.3 * U(g) : 30.0 * U(g));
    double qn = 0;
    for (int i = 3; i < 7; ++i) qn += (double)x[i] * x[i];
    for (int i = 3; i < 7; ++i) x[i] = (float)(x[i] / std::sqrt(qn));
    const HalfInvT<float> A = half_step_inverse(Ps[e], sc.h2);
    for (int t = 0; t < T; ++t) {
      if (t % K == 0)
        for (int i = 0; i < D; ++i) ckpt[((size_t)(t / K) * Dio + i) * E + e] = x[i];
      float a[N], fcmd[N], gcmd[6];
      for (int i = 0; i < N; ++i) a[i] = act[((size_t)t * n_max + i) * E + e];
      thrust_command<N>(cc, a, fcmd);
      command_wrench<N>(cc, fcmd, gcmd);
      control_step<N, LAG>(x, Ps[e], A, cc, fcmd, gcmd, sc, S, cc.rho_s);
    }
  }
  const int64_t Ep = (E + 255) / 256 * 256;
  struct Out {
    std::vector<float> gact, gth, gx0;
  };
  auto run = [&](int form) {
    Out o{std::vector<float>((size_t)T * n_max * E, NAN), std::vector<float>((size_t)19 * E, NAN),
          std::vector<float>((size_t)Dio * E, NAN)};
    const int rows = form == 2 ? T * S : std::min(K, T) * S;
    std::vector<float> segbuf((size_t)rows * D * Ep, NAN);
    AdjArgs a;
    std::memset(&a, 0, sizeof a);
    a.Ep = Ep;
    a.E = E;
    a.seg_start = 0;
    a.seg_len = E;
    a.actions = act.data();
    a.n_max = n_max;
    a.D = Dio;
    a.T = T;
    a.substeps = S;
    a.ckpt_every = K;
    a.dt = dt;
    a.ckpt = ckpt.data();
    a.gtraj = gtraj.data();
    a.gact = o.gact.data();
    a.gtheta = o.gth.data();
    a.gx0 = o.gx0.data();
    a.segbuf = segbuf.data();
    a.zb = 0.0f;
    a.recomputed = form == 2;
    for (int e = 0; e < E; ++e) {
      const HalfInvT<float> A = half_step_inverse(Ps[e], sc.h2);
      ThetaBar<float> thb;
      theta_bar_zero(thb);
      if (form == 0) {
        adj_bwd_env<N, LAG, false>(a, cc, Ps[e], sc, A, e, e, thb);
      } else if (form == 3) {
        adj_bwd_env<N, LAG, false, true>(a, cc, Ps[e], sc, A, e, e, thb);
      } else if (form == 1) {
        adj_bwd_env_factored<N, LAG>(a, cc, Ps[e], sc, A, e, e);
      } else {
        for (int seg = 0; seg < nseg; ++seg) {
          float x[D];
          for (int i = 0; i < D; ++i) x[i] = ckpt[((size_t)seg * Dio + i) * E + e];
          recompute_segment<N, LAG>(a, cc, Ps[e], A, sc, x, seg * K, std::min(T, seg * K + K), 0,
                                    e, e);
        }
        adj_bwd_env<N, LAG, true>(a, cc, Ps[e], sc, A, e, e, thb);
      }
    }
    return o;
  };
  const Out cur = run(0), fac = run(1), whole = run(2), pre = run(3);
  auto same = [](const std::vector<float>& x, const std::vector<float>& y) {
    return x.size() == y.size() && std::memcmp(x.data(), y.data(), x.size() * 4) == 0;
  };
  auto finite = [](const std::vector<float>& x) {
    for (float v : x)
      if (!std::isfinite(v)) return false;
    return true;
  };
  const bool ok = same(cur.gact, fac.gact) && same(cur.gth, fac.gth) && same(cur.gx0, fac.gx0) &&
                  same(cur.gact, whole.gact) && same(cur.gth, whole.gth) &&
                  same(cur.gx0, whole.gx0) && same(cur.gact, pre.gact) &&
                  same(cur.gth, pre.gth) && same(cur.gx0, pre.gx0) && finite(cur.gact) &&
                  finite(cur.gth) &&
                  finite(cur.gx0);
  std::printf("N=%d lag=%d E=%d T=%d K=%d S=%d: %s\n", N, (int)LAG, E, T, K, S,
              ok ? "current = factored = whole = prefetching, bitwise, all finite" : "MISMATCH");
  if (!ok) ++failures;
}

}  // namespace

int main() {
  check<8, true>(1, 300, 6, 8, 3, 1, 0.005f);     // one segment: the one-wave instantiation's case
  check<8, true>(2, 257, 13, 4, 3, 1, 0.005f);
  check<8, false>(3, 300, 6, 8, 3, 1, 0.005f);
  check<6, true>(4, 200, 10, 3, 4, 1, 0.005f);
  check<6, false>(5, 300, 16, 8, 1, 0, 0.01f);    // the tracking-loss workload's shape
  check<1, true>(6, 65, 7, 3, 2, 1, 0.02f);
  std::printf("%d failures\n", failures);
  return failures ? 1 : 0;
}
