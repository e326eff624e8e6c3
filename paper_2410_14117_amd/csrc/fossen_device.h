// fossen_device.h -- per-env Fossen right-hand side and RK4 sub-step, FP32,
// everything in registers.  Included by the kernel translation units only.
//
// State x = [p(3), q(4), nu(6), f(N if LAG)]; see include/mg.h for the layout.
// The equation is MarineGym's Eq. (1) (Sec. II) solved for nu':
//   nu' = M^-1 (tau - C(nu) nu - D(nu) nu - g(q)),   M = M_RB + M_A
// using the Kirchhoff form of the Coriolis term, C(nu) nu = [w x a ; v x a + w x b]
// with [a; b] = M nu (the same vector as the skew-symmetric C_RB + C_A matrix
// times nu, at a fraction of the work), and the structure of M for diagonal
// I_g, M_A and r_g on the z axis: M and M^-1 couple only (u,q) and (v,p).
#pragma once

#include "mg_internal.h"

namespace mg {

// Per-env constants held in registers for the whole launch.
struct EnvConst {
  float Muu, Mvv, Mww, Mpp, Mqq, Mrr, Muq, Mvp;
  float Iuu, Ivv, Iww, Ipp, Iqq, Irr, Iuq, Ivp;
  float dl[6], dq[6];
  float wmb, hz;
};

__device__ __forceinline__ EnvConst load_env_const(const float* __restrict__ der, int64_t Ep,
                                                   int64_t j) {
  EnvConst P;
  P.Muu = der[kMuu * Ep + j]; P.Mvv = der[kMvv * Ep + j]; P.Mww = der[kMww * Ep + j];
  P.Mpp = der[kMpp * Ep + j]; P.Mqq = der[kMqq * Ep + j]; P.Mrr = der[kMrr * Ep + j];
  P.Muq = der[kMuq * Ep + j]; P.Mvp = der[kMvp * Ep + j];
  P.Iuu = der[kIuu * Ep + j]; P.Ivv = der[kIvv * Ep + j]; P.Iww = der[kIww * Ep + j];
  P.Ipp = der[kIpp * Ep + j]; P.Iqq = der[kIqq * Ep + j]; P.Irr = der[kIrr * Ep + j];
  P.Iuq = der[kIuq * Ep + j]; P.Ivp = der[kIvp * Ep + j];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    P.dl[i] = der[(kDL + i) * Ep + j];
    P.dq[i] = der[(kDQ + i) * Ep + j];
  }
  P.wmb = der[kWmB * Ep + j];
  P.hz = der[kHz * Ep + j];
  return P;
}

template <int N, bool LAG>
struct Dims {
  static constexpr int D = 13 + (LAG ? N : 0);
};

// Commanded thrust from a throttle frame (Eq. (3)): clamp to [-1,1], then
// f_max a (linear) or f_max a|a| (quadratic).
template <int N>
__device__ __forceinline__ void thrust_command(const ClassConst& cc, const float (&a)[N],
                                               float (&fcmd)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    // fminf/fmaxf would turn a NaN throttle into a number; keep NaN flowing
    float ai = a[i] > 1.0f ? 1.0f : (a[i] < -1.0f ? -1.0f : a[i]);
    fcmd[i] = cc.thr_map ? cc.f_max * ai * fabsf(ai) : cc.f_max * ai;
  }
}

// Wrench of the commanded thrust, B f_cmd (once per control step).
template <int N>
__device__ __forceinline__ void command_wrench(const ClassConst& cc, const float (&fcmd)[N],
                                               float (&gcmd)[6]) {
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    float s = cc.B[k][0] * fcmd[0];
#pragma unroll
    for (int i = 1; i < N; ++i) s = fmaf(cc.B[k][i], fcmd[i], s);
    gcmd[k] = s;
  }
}

// Right-hand side of the 13 rigid-body states x = [p, q, nu] for a given
// body wrench tau.  Written as fused multiply-add chains:
//   p'  = R(q) v, as v + q_w t + q_v x t with t = 2 q_v x v (the same value as
//         the unit-quaternion rotation matrix times v, for any q)
//   xd[3..6] = q (x) (0, w)   -- TWICE q'; the caller applies the 1/2
//   nu' = M^-1 (tau - C(nu) nu - D(nu) nu - g(q)),  with
//         C(nu) nu = [w x a ; v x a + w x b], [a; b] = M nu (Kirchhoff form of
//         the skew-symmetric C_RB + C_A), D diagonal linear + quadratic,
//         g = -[(W-B) k ; h x k], k = R(q)^T e3, h = (0, 0, W z_g - B z_b).
// xd may not alias x.
__device__ __forceinline__ void rhs_core(const float* x, float* xd, const EnvConst& P,
                                         const float (&tau)[6]) {
  const float qw = x[3], qx = x[4], qy = x[5], qz = x[6];
  const float u = x[7], v = x[8], w = x[9], p = x[10], q = x[11], r = x[12];

  // kinematics
  const float x2 = qx + qx, y2 = qy + qy, z2 = qz + qz;
  const float t0 = fmaf(y2, w, -z2 * v);
  const float t1 = fmaf(z2, u, -x2 * w);
  const float t2 = fmaf(x2, v, -y2 * u);
  xd[0] = fmaf(-qz, t1, fmaf(qy, t2, fmaf(qw, t0, u)));
  xd[1] = fmaf(-qx, t2, fmaf(qz, t0, fmaf(qw, t1, v)));
  xd[2] = fmaf(-qy, t0, fmaf(qx, t1, fmaf(qw, t2, w)));
  xd[3] = -fmaf(qx, p, fmaf(qy, q, qz * r));
  xd[4] = fmaf(-qz, q, fmaf(qy, r, qw * p));
  xd[5] = fmaf(-qx, r, fmaf(qz, p, qw * q));
  xd[6] = fmaf(-qy, p, fmaf(qx, q, qw * r));
  // k = R^T e3, the third row of R(q)
  const float k0 = fmaf(x2, qz, -y2 * qw);
  const float k1 = fmaf(y2, qz, x2 * qw);
  const float k2 = fmaf(-y2, qy, fmaf(-x2, qx, 1.0f));

  // [a; b] = M nu
  const float au = fmaf(P.Muq, q, P.Muu * u), av = fmaf(P.Mvp, p, P.Mvv * v), aw = P.Mww * w;
  const float bp = fmaf(P.Mpp, p, P.Mvp * v), bq = fmaf(P.Mqq, q, P.Muq * u), br = P.Mrr * r;
  // damping coefficients d_L + d_Q |nu|
  const float e0 = fmaf(P.dq[0], fabsf(u), P.dl[0]);
  const float e1 = fmaf(P.dq[1], fabsf(v), P.dl[1]);
  const float e2 = fmaf(P.dq[2], fabsf(w), P.dl[2]);
  const float e3 = fmaf(P.dq[3], fabsf(p), P.dl[3]);
  const float e4 = fmaf(P.dq[4], fabsf(q), P.dl[4]);
  const float e5 = fmaf(P.dq[5], fabsf(r), P.dl[5]);
  // residual tau - C nu - D nu - g
  const float r0 = fmaf(-e0, u, fmaf(P.wmb, k0, fmaf(-q, aw, fmaf(r, av, tau[0]))));
  const float r1 = fmaf(-e1, v, fmaf(P.wmb, k1, fmaf(-r, au, fmaf(p, aw, tau[1]))));
  const float r2 = fmaf(-e2, w, fmaf(P.wmb, k2, fmaf(-p, av, fmaf(q, au, tau[2]))));
  const float r3 = fmaf(-e3, p, fmaf(-P.hz, k1,
                   fmaf(r, bq, fmaf(-q, br, fmaf(w, av, fmaf(-v, aw, tau[3]))))));
  const float r4 = fmaf(-e4, q, fmaf(P.hz, k0,
                   fmaf(p, br, fmaf(-r, bp, fmaf(u, aw, fmaf(-w, au, tau[4]))))));
  const float r5 = fmaf(-e5, r, fmaf(q, bp, fmaf(-p, bq, fmaf(v, au, fmaf(-u, av, tau[5])))));
  // nu' = M^-1 r
  xd[7] = fmaf(P.Iuq, r4, P.Iuu * r0);
  xd[8] = fmaf(P.Ivp, r3, P.Ivv * r1);
  xd[9] = P.Iww * r2;
  xd[10] = fmaf(P.Ipp, r3, P.Ivp * r1);
  xd[11] = fmaf(P.Iqq, r4, P.Iuq * r0);
  xd[12] = P.Irr * r5;
}

// One classical RK4 sub-step (c = 0, 1/2, 1/2, 1; b = 1/6, 1/3, 1/3, 1/6) of
// the full state [p, q, nu, f], then q <- q / |q|.
//
// The thruster states enter only through the wrench B f and obey the linear
// lag f' = (f_cmd - f) / tau with f_cmd held, so their RK4 stage values are
// f_cmd + sigma_i (f - f_cmd) exactly (class constants), the stage wrenches
// are B f_cmd + sigma_i B (f - f_cmd), and the sub-step maps f - f_cmd to
// rho (f - f_cmd): the same discrete map as generic RK4 on the lag states,
// with one allocation product per sub-step instead of four.  Without a lag
// the wrench is the command wrench B f_cmd throughout.
template <int N, bool LAG>
__device__ __forceinline__ void rk4_substep(float* x, const EnvConst& P, const ClassConst& cc,
                                            const float (&fcmd)[N], const float (&gcmd)[6],
                                            float dt) {
  const float h2 = 0.5f * dt, h6 = dt * (1.0f / 6.0f);
  float df[N], dg[6], tau[6];
  if constexpr (LAG) {
#pragma unroll
    for (int i = 0; i < N; ++i) df[i] = x[13 + i] - fcmd[i];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      float s = cc.B[k][0] * df[0];
#pragma unroll
      for (int i = 1; i < N; ++i) s = fmaf(cc.B[k][i], df[i], s);
      dg[k] = s;
      tau[k] = gcmd[k] + s;
    }
  } else {
#pragma unroll
    for (int k = 0; k < 6; ++k) tau[k] = gcmd[k];
  }
  // stage / combination factors; the quaternion rows of rhs_core are 2 q'
  auto fac = [](int i, float f) { return (i >= 3 && i < 7) ? 0.5f * f : f; };
  float k[13], X[13], acc[13];
  rhs_core(x, k, P, tau);
#pragma unroll
  for (int i = 0; i < 13; ++i) {
    acc[i] = k[i];
    X[i] = fmaf(fac(i, h2), k[i], x[i]);
  }
  if constexpr (LAG) {
#pragma unroll
    for (int j = 0; j < 6; ++j) tau[j] = fmaf(cc.sigma2, dg[j], gcmd[j]);
  }
  rhs_core(X, k, P, tau);
#pragma unroll
  for (int i = 0; i < 13; ++i) {
    acc[i] = fmaf(2.0f, k[i], acc[i]);
    X[i] = fmaf(fac(i, h2), k[i], x[i]);
  }
  if constexpr (LAG) {
#pragma unroll
    for (int j = 0; j < 6; ++j) tau[j] = fmaf(cc.sigma3, dg[j], gcmd[j]);
  }
  rhs_core(X, k, P, tau);
#pragma unroll
  for (int i = 0; i < 13; ++i) {
    acc[i] = fmaf(2.0f, k[i], acc[i]);
    X[i] = fmaf(fac(i, dt), k[i], x[i]);
  }
  if constexpr (LAG) {
#pragma unroll
    for (int j = 0; j < 6; ++j) tau[j] = fmaf(cc.sigma4, dg[j], gcmd[j]);
  }
  rhs_core(X, k, P, tau);
#pragma unroll
  for (int i = 0; i < 13; ++i) x[i] = fmaf(fac(i, h6), acc[i] + k[i], x[i]);
  if constexpr (LAG) {
#pragma unroll
    for (int i = 0; i < N; ++i) x[13 + i] = fmaf(cc.rho, df[i], fcmd[i]);
  }
  const float n2 = x[3] * x[3] + x[4] * x[4] + x[5] * x[5] + x[6] * x[6];
  const float inv = rsqrtf(n2);
  x[3] *= inv;
  x[4] *= inv;
  x[5] *= inv;
  x[6] *= inv;
}

}  // namespace mg
