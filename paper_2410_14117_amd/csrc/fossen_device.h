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

// x' = f(x).  xd may not alias x.
template <int N, bool LAG>
__device__ __forceinline__ void rhs(const float* x, float* xd, const EnvConst& P,
                                    const ClassConst& cc, const float (&fcmd)[N]) {
  const float qw = x[3], qx = x[4], qy = x[5], qz = x[6];
  const float u = x[7], v = x[8], w = x[9], p = x[10], q = x[11], r = x[12];

  // rotation body -> NED (unit-quaternion formula, stage quaternion as is)
  const float xx = qx * qx, yy = qy * qy, zz = qz * qz;
  const float xy = qx * qy, xz = qx * qz, yz = qy * qz;
  const float wx = qw * qx, wy = qw * qy, wz = qw * qz;
  const float R00 = 1.0f - 2.0f * (yy + zz), R01 = 2.0f * (xy - wz), R02 = 2.0f * (xz + wy);
  const float R10 = 2.0f * (xy + wz), R11 = 1.0f - 2.0f * (xx + zz), R12 = 2.0f * (yz - wx);
  const float R20 = 2.0f * (xz - wy), R21 = 2.0f * (yz + wx), R22 = 1.0f - 2.0f * (xx + yy);

  // kinematics
  xd[0] = R00 * u + R01 * v + R02 * w;
  xd[1] = R10 * u + R11 * v + R12 * w;
  xd[2] = R20 * u + R21 * v + R22 * w;
  const float hp = 0.5f * p, hq = 0.5f * q, hr = 0.5f * r;
  xd[3] = -(qx * hp + qy * hq + qz * hr);
  xd[4] = qw * hp + qy * hr - qz * hq;
  xd[5] = qw * hq + qz * hp - qx * hr;
  xd[6] = qw * hr + qx * hq - qy * hp;

  // thrust -> body wrench
  const float* th = LAG ? x + 13 : fcmd;
  float tau[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    float s = cc.B[k][0] * th[0];
#pragma unroll
    for (int i = 1; i < N; ++i) s += cc.B[k][i] * th[i];
    tau[k] = s;
  }

  // [a; b] = M nu
  const float au = P.Muu * u + P.Muq * q, av = P.Mvv * v + P.Mvp * p, aw = P.Mww * w;
  const float bp = P.Mvp * v + P.Mpp * p, bq = P.Muq * u + P.Mqq * q, br = P.Mrr * r;
  // C(nu) nu = [w x a ; v x a + w x b]
  const float c0 = q * aw - r * av;
  const float c1 = r * au - p * aw;
  const float c2 = p * av - q * au;
  const float c3 = (v * aw - w * av) + (q * br - r * bq);
  const float c4 = (w * au - u * aw) + (r * bp - p * br);
  const float c5 = (u * av - v * au) + (p * bq - q * bp);
  // D(nu) nu, diagonal linear + quadratic
  const float d0 = (P.dl[0] + P.dq[0] * fabsf(u)) * u;
  const float d1 = (P.dl[1] + P.dq[1] * fabsf(v)) * v;
  const float d2 = (P.dl[2] + P.dq[2] * fabsf(w)) * w;
  const float d3 = (P.dl[3] + P.dq[3] * fabsf(p)) * p;
  const float d4 = (P.dl[4] + P.dq[4] * fabsf(q)) * q;
  const float d5 = (P.dl[5] + P.dq[5] * fabsf(r)) * r;
  // restoring g = -[(W-B) k ; h x k], k = R^T e3 = (R20, R21, R22), h = (0, 0, hz)
  const float r0 = tau[0] - c0 - d0 + P.wmb * R20;
  const float r1 = tau[1] - c1 - d1 + P.wmb * R21;
  const float r2 = tau[2] - c2 - d2 + P.wmb * R22;
  const float r3 = tau[3] - c3 - d3 - P.hz * R21;
  const float r4 = tau[4] - c4 - d4 + P.hz * R20;
  const float r5 = tau[5] - c5 - d5;
  // nu' = M^-1 r
  xd[7] = P.Iuu * r0 + P.Iuq * r4;
  xd[8] = P.Ivv * r1 + P.Ivp * r3;
  xd[9] = P.Iww * r2;
  xd[10] = P.Ivp * r1 + P.Ipp * r3;
  xd[11] = P.Iuq * r0 + P.Iqq * r4;
  xd[12] = P.Irr * r5;
  if constexpr (LAG) {
#pragma unroll
    for (int i = 0; i < N; ++i) xd[13 + i] = (fcmd[i] - x[13 + i]) * cc.inv_tau;
  }
}

// One classical RK4 sub-step (c = 0, 1/2, 1/2, 1; b = 1/6, 1/3, 1/3, 1/6),
// then q <- q / |q|.
template <int N, bool LAG>
__device__ __forceinline__ void rk4_substep(float* x, const EnvConst& P, const ClassConst& cc,
                                            const float (&fcmd)[N], float dt) {
  constexpr int D = Dims<N, LAG>::D;
  const float h2 = 0.5f * dt, h6 = dt * (1.0f / 6.0f);
  float k[D], X[D], acc[D];
  rhs<N, LAG>(x, k, P, cc, fcmd);
#pragma unroll
  for (int i = 0; i < D; ++i) {
    acc[i] = k[i];
    X[i] = x[i] + h2 * k[i];
  }
  rhs<N, LAG>(X, k, P, cc, fcmd);
#pragma unroll
  for (int i = 0; i < D; ++i) {
    acc[i] += 2.0f * k[i];
    X[i] = x[i] + h2 * k[i];
  }
  rhs<N, LAG>(X, k, P, cc, fcmd);
#pragma unroll
  for (int i = 0; i < D; ++i) {
    acc[i] += 2.0f * k[i];
    X[i] = x[i] + dt * k[i];
  }
  rhs<N, LAG>(X, k, P, cc, fcmd);
#pragma unroll
  for (int i = 0; i < D; ++i) x[i] += h6 * (acc[i] + k[i]);
  const float n2 = x[3] * x[3] + x[4] * x[4] + x[5] * x[5] + x[6] * x[6];
  const float inv = rsqrtf(n2);
  x[3] *= inv;
  x[4] *= inv;
  x[5] *= inv;
  x[6] *= inv;
}

}  // namespace mg
