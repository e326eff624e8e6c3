// kernels_task.hip -- Gym-style task step of Sec. III: one control step of
// the fused sub-step loop followed by the task epilogue (the error of Eq. (4),
// episode end, automatic reset, the observation of Eq. (2)), or the
// observation alone.  One env per lane; the epilogue works in FP64 from the
// FP32 state and writes FP32.
#include "fossen_device.h"

namespace mg {

namespace {

constexpr double kPi = 3.1415926535897932384626433832795;

// Reference point p_r and the horizontal direction (vx, vy) of the reference
// heading, given sin and cos of the curve parameter s = omega t + phase.  For
// the circle and the helix the reference velocity is omega R (-sin s, cos s);
// for the lemniscate of Bernoulli R (cos s, sin s cos s) / (1 + sin^2 s) it is
// omega R (-sin s (3 - sin^2 s), 1 - 3 sin^2 s) / (1 + sin^2 s)^2 (the positive
// factor R / (1 + sin^2 s)^2 drops out of the direction).  Station keeping:
// the centre, headed along the target yaw.
__device__ __forceinline__ void reference(const TaskConst& tc, const double (&c)[3], double yaw,
                                          double t, double sn, double cs, double (&pr)[3],
                                          double& vx, double& vy) {
  if (tc.task == 0) {
    pr[0] = c[0];
    pr[1] = c[1];
    pr[2] = c[2];
    float sy, cy;
    sincosf((float)yaw, &sy, &cy);
    vx = cy;
    vy = sy;
    return;
  }
  if (tc.task == 3) {
    const double s2 = mul_nc(sn, sn), inv = 1.0 / (1.0 + s2);
    pr[0] = c[0] + tc.R * cs * inv;
    pr[1] = c[1] + tc.R * sn * cs * inv;
    pr[2] = c[2];
    vx = -tc.omega * sn * (3.0 - s2);
    vy = tc.omega * (1.0 - 3.0 * s2);
  } else {
    pr[0] = c[0] + tc.R * cs;
    pr[1] = c[1] + tc.R * sn;
    pr[2] = c[2] + (tc.task == 2 ? tc.climb * t : 0.0);
    vx = -tc.omega * sn;
    vy = tc.omega * cs;
  }
}

// Writes the observation of Eq. (2) of the state x at episode step k, given
// sin and cos of the curve parameter at that time.  The heading error
// wrap(yaw - yaw_r) is the signed angle from the reference direction (vx, vy)
// to the body's horizontal heading h = R(q) e1 (parallel to (cos yaw, sin yaw)
// while |pitch| < 90 deg), one atan2 per point; the curve parameters of the
// look-ahead points follow one another by the rotation (cos, sin)(omega dl).
__device__ __forceinline__ void observe(const TaskConst& tc, const float* x, const double (&c)[3],
                                        double yaw, int32_t k, double sn, double cs, float* obs,
                                        int64_t E) {
  // ZYX roll and pitch from the third row of R(q): roll = atan2(R32, R33),
  // pitch = atan2(-R31, |(R32, R33)|) (well conditioned at any pitch, unlike
  // asin(-R31) near +-90 deg)
  const float w = x[3], qx = x[4], qy = x[5], qz = x[6];
  const float r32 = 2.0f * (w * qx + qy * qz), r33 = 1.0f - 2.0f * (qx * qx + qy * qy);
  const float r31 = 2.0f * (qx * qz - w * qy);
  float roll = atan2f(r32, r33);
  if (roll <= -3.14159265f) roll = 3.14159265f;
  const float pitch = atan2f(-r31, sqrtf(r32 * r32 + r33 * r33));
  const double hx = 1.0 - 2.0 * ((double)qy * qy + (double)qz * qz);
  const double hy = 2.0 * ((double)qx * qy + (double)w * qz);
  const double t = k * tc.dtc;
  const int m = tc.task == 0 ? 1 : tc.m;
  for (int i = 0; i < m; ++i) {
    const double sn1 = fma(sn, tc.cdl, cs * tc.sdl);
    cs = fma(cs, tc.cdl, -sn * tc.sdl);
    sn = sn1;
    double pr[3], vx, vy;
    reference(tc, c, yaw, fma((double)(i + 1), tc.dl, t), sn, cs, pr, vx, vy);
    float herr = atan2f((float)(hy * vx - hx * vy), (float)(hx * vx + hy * vy));
    if (herr <= -3.14159265f) herr = 3.14159265f;
    float* o = obs + (int64_t)(6 * i) * E;
    o[0] = (float)(x[0] - pr[0]);
    o[E] = (float)(x[1] - pr[1]);
    o[2 * E] = (float)(x[2] - pr[2]);
    o[3 * E] = roll;
    o[4 * E] = pitch;
    o[5 * E] = herr;
  }
  float* o = obs + (int64_t)(6 * m) * E;
#pragma unroll
  for (int i = 0; i < 6; ++i) o[i * E] = x[7 + i];
}

// sin and cos of the curve parameter s = omega t + phase: s is formed and
// reduced to [-pi, pi] in FP64, then evaluated in FP32 (errors ~1e-7, well
// inside the observation's FP32 output).
__device__ __forceinline__ void curve_sincos(const TaskConst& tc, double t, double phase,
                                             double& sn, double& cs) {
  if (tc.task == 0) {
    sn = 0.0;
    cs = 1.0;
    return;
  }
  const double s = fma(tc.omega, t, phase);
  const double r = s - (2.0 * kPi) * rint(s * (0.5 / kPi));
  float sf, cf;
  sincosf((float)r, &sf, &cf);
  sn = sf;
  cs = cf;
}

}  // namespace

// Held to three resident waves per SIMD (at most 168 VGPRs), the step kernel's
// occupancy: left to itself the compiler gives the 8-thruster lag variant 170
// registers for the epilogue, which leaves room for two waves only.
template <int N, bool LAG>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3)))
k_task(const TaskArgs a, const ClassConst cc, const TaskConst tc) {
  constexpr int D = Dims<N, LAG>::D;
  const int64_t local = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (local >= a.seg_len) return;
  if (!MG_CHECK(a, a.seg_start + a.seg_len <= a.Ep, kDbgSegment)) return;
  const int64_t j = a.seg_start + local;
  const int64_t c = a.perm ? (int64_t)a.perm[j] : j;
  if (!MG_CHECK(a, c >= 0 && c < a.dbg.cols, kDbgColumn)) return;
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
  // sin and cos of the curve parameter at the current episode time
  double sn, cs;
  curve_sincos(tc, k * tc.dtc, phase, sn, cs);
  if (a.actions) {
    bool finite = true;
#pragma unroll
    for (int i = 0; i < D; ++i) finite = finite && isfinite(x[i]);
    double pr[3], vx, vy;
    reference(tc, cen, yaw, k * tc.dtc, sn, cs, pr, vx, vy);
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
      curve_sincos(tc, 0.0, phase, sn, cs);
      uint8_t fl = (uint8_t)(a.flags[j] & kFlagNotSPD);
      if (a.reset_mult)
        fl = set_env_params(*a.nominal, a.reset_mult + c, a.E, false, a.params, a.derived, a.Ep,
                            j) ? 0 : kFlagNotSPD;
      a.flags[j] = fl;
    }
#pragma unroll
    for (int i = 0; i < D; ++i) a.state[i * a.Ep + j] = x[i];
    a.task_k[j] = k;
  }
  observe(tc, x, cen, yaw, k, sn, cs, a.obs + c, a.E);
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
