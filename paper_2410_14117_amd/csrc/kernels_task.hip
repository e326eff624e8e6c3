// kernels_task.hip -- Gym-style task step of Sec. III: one control step of
// the fused sub-step loop followed by the task epilogue (the error of Eq. (4),
// episode end, automatic reset, the observation of Eq. (2)), or the
// observation alone.  One env per lane; the epilogue works in FP64 from the
// FP32 state and writes FP32.
#include "fossen_device.h"

namespace mg {

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kPi = 3.1415926535897932384626433832795;

// Angle in (-pi, pi].
__device__ __forceinline__ double wrap_pi(double a) {
  double r = a - kTwoPi * rint(a / kTwoPi);
  if (r <= -kPi) r += kTwoPi;
  if (r > kPi) r -= kTwoPi;
  return r;
}

// Reference point and heading at episode time t.  Curve parameter
// s = omega t + phase; the heading follows the horizontal reference velocity,
// which is omega (-sin s, cos s) R for the circle and the helix and, for the
// lemniscate of Bernoulli R (cos s, sin s cos s) / (1 + sin^2 s),
// omega R (-sin s (3 - sin^2 s), 1 - 3 sin^2 s) / (1 + sin^2 s)^2.
__device__ __forceinline__ void reference(const TaskConst& tc, const double (&c)[3], double phase,
                                          double yaw, double t, double (&pr)[3], double& psi) {
  if (tc.task == 0) {
    pr[0] = c[0];
    pr[1] = c[1];
    pr[2] = c[2];
    psi = yaw;
    return;
  }
  double sn, cs;
  sincos(fma(tc.omega, t, phase), &sn, &cs);
  if (tc.task == 3) {
    const double s2 = sn * sn, inv = 1.0 / (1.0 + s2);
    pr[0] = c[0] + tc.R * cs * inv;
    pr[1] = c[1] + tc.R * sn * cs * inv;
    pr[2] = c[2];
    psi = atan2(tc.omega * (1.0 - 3.0 * s2), -tc.omega * sn * (3.0 - s2));
  } else {
    pr[0] = c[0] + tc.R * cs;
    pr[1] = c[1] + tc.R * sn;
    pr[2] = c[2] + (tc.task == 2 ? tc.climb * t : 0.0);
    psi = atan2(tc.omega * cs, -tc.omega * sn);
  }
}

// Writes the observation of Eq. (2) of the state x at episode step k.
__device__ __forceinline__ void observe(const TaskConst& tc, const float* x, const double (&c)[3],
                                        double phase, double yaw, int32_t k, float* obs,
                                        int64_t E) {
  const double w = x[3], qx = x[4], qy = x[5], qz = x[6];
  // ZYX roll, pitch, yaw of the unit quaternion
  const double roll = atan2(2.0 * (w * qx + qy * qz), 1.0 - 2.0 * (qx * qx + qy * qy));
  const double sp = fmin(1.0, fmax(-1.0, 2.0 * (w * qy - qz * qx)));
  const double pitch = asin(sp);
  const double head = atan2(2.0 * (w * qz + qx * qy), 1.0 - 2.0 * (qy * qy + qz * qz));
  const double t = k * tc.dtc;
  const int m = tc.task == 0 ? 1 : tc.m;
  for (int i = 0; i < m; ++i) {
    double pr[3], psi;
    reference(tc, c, phase, yaw, tc.task == 0 ? t : fma((double)(i + 1), tc.dl, t), pr, psi);
    float* o = obs + (int64_t)(6 * i) * E;
    o[0] = (float)(x[0] - pr[0]);
    o[E] = (float)(x[1] - pr[1]);
    o[2 * E] = (float)(x[2] - pr[2]);
    o[3 * E] = (float)wrap_pi(roll);
    o[4 * E] = (float)wrap_pi(pitch);
    o[5 * E] = (float)wrap_pi(head - psi);
  }
  float* o = obs + (int64_t)(6 * m) * E;
#pragma unroll
  for (int i = 0; i < 6; ++i) o[i * E] = x[7 + i];
}

}  // namespace

template <int N, bool LAG>
__global__ void __launch_bounds__(kBlock) k_task(const TaskArgs a, const ClassConst cc,
                                                 const TaskConst tc) {
  constexpr int D = Dims<N, LAG>::D;
  const int64_t local = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (local >= a.seg_len) return;
  const int64_t j = a.seg_start + local;
  const int64_t c = a.perm ? (int64_t)a.perm[j] : j;
  float x[D];
#pragma unroll
  for (int i = 0; i < D; ++i) x[i] = a.state[i * a.Ep + j];
  int32_t k = a.task_k[j];
  if (a.actions) {
    const EnvConst P = load_env_const(a.derived, a.Ep, j);
    const StepConstT<float> sc = make_step_const(cc, a.dt);
    const HalfInvT<float> A = half_step_inverse(P, sc.h2);
    float act[N], fcmd[N], gcmd[6];
#pragma unroll
    for (int i = 0; i < N; ++i) act[i] = a.actions[i * a.E + c];
    thrust_command<N>(cc, act, fcmd);
    command_wrench<N>(cc, fcmd, gcmd);
    control_step<N, LAG>(x, P, A, cc, fcmd, gcmd, sc, a.substeps,
                         a.substeps == 1 ? cc.rho : cc.rho_s);
    k += 1;
  }
  // the task's per-env data is read after the sub-steps, so that it does not
  // occupy registers across them
  const double cen[3] = {a.task_f[j], a.task_f[a.Ep + j], a.task_f[2 * a.Ep + j]};
  const double phase = a.task_f[3 * a.Ep + j], yaw = a.task_f[4 * a.Ep + j];
  if (a.actions) {
    bool finite = true;
#pragma unroll
    for (int i = 0; i < D; ++i) finite = finite && isfinite(x[i]);
    double pr[3], psi;
    reference(tc, cen, phase, yaw, k * tc.dtc, pr, psi);
    const double dx = x[0] - pr[0], dy = x[1] - pr[1], dz = x[2] - pr[2];
    const double e = sqrt(dx * dx + dy * dy + dz * dz);
    const bool term = !finite || (tc.emax > 0.0 && !(e <= tc.emax));
    const int32_t d = term ? 1 : (k >= tc.L ? 2 : 0);
    if (a.err) a.err[c] = (float)e;
    if (a.done) a.done[c] = d;
    if (d) {
#pragma unroll
      for (int i = 0; i < D; ++i)
        x[i] = a.reset_state ? a.reset_state[i * a.E + c] : (i == 3 ? 1.0f : 0.0f);
      k = 0;
      if (a.reset_mult)
        set_env_params(*a.nominal, a.reset_mult + c, a.E, false, a.params, a.derived, a.Ep, j);
    }
#pragma unroll
    for (int i = 0; i < D; ++i) a.state[i * a.Ep + j] = x[i];
    a.task_k[j] = k;
  }
  observe(tc, x, cen, phase, yaw, k, a.obs + c, a.E);
}

template <int N, bool LAG>
static hipError_t launch_task_t(const ClassConst& cc, const TaskConst& tc, const TaskArgs& a,
                                hipStream_t s) {
  const int64_t nblk = (a.seg_len + kBlock - 1) / kBlock;
  if (nblk == 0) return hipSuccess;
  hipLaunchKernelGGL((k_task<N, LAG>), dim3((unsigned)nblk), dim3(kBlock), 0, s, a, cc, tc);
  return hipGetLastError();
}

hipError_t launch_task(const ClassConst& cc, const TaskConst& tc, const TaskArgs& a,
                       hipStream_t s) {
  const bool lag = cc.lag != 0;
#define MG_CASE(n)                                                                   \
  case n:                                                                            \
    return lag ? launch_task_t<n, true>(cc, tc, a, s) : launch_task_t<n, false>(cc, tc, a, s);
  switch (cc.n_thr) {
    MG_CASE(1) MG_CASE(2) MG_CASE(3) MG_CASE(4) MG_CASE(5) MG_CASE(6) MG_CASE(7) MG_CASE(8)
    default:
      return hipErrorInvalidValue;
  }
#undef MG_CASE
}

}  // namespace mg
