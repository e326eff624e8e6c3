// fossen_adjoint.h -- reverse mode of the RK4 sub-step of fossen_device.h:
// vector-Jacobian products of the right-hand side and of one whole sub-step
// (stages, combination, quaternion renormalisation, closed-form lag stages),
// with respect to the state, the commanded thrust and the per-env
// hydrodynamic parameters theta = (M_A(6), D_L(6), D_Q(6), B).
//
// Everything is exact for the discrete map the forward kernels compute; the
// forward intermediates are recomputed from the sub-step input.
#pragma once

#include "fossen_device.h"

namespace mg {

// Adjoints of the parameter-dependent constants: diagonal of M (M_A enters
// there; the off-diagonal m z_g terms do not depend on theta), the damping
// diagonals, W - B and h_z = W z_g - B z_b.
template <class T>
struct ThetaBar {
  T ma[6], dl[6], dq[6], wmb, hz;
};

template <class T>
__host__ __device__ __forceinline__ void theta_bar_zero(ThetaBar<T>& t) {
#pragma unroll
  for (int i = 0; i < 6; ++i) t.ma[i] = t.dl[i] = t.dq[i] = T(0);
  t.wmb = t.hz = T(0);
}

// The same adjoints held in LDS, [20][kBlock] floats (slot k of a lane at
// col + k kBlock), for the two-wave trajectory-reading sweep, which has 256
// registers and would otherwise spill inside the sub-step VJP: each
// += / -= is a load, the same operation and a store, so the sums are those of
// ThetaBar, bitwise.  theta_bar_fence, a compiler-only memory barrier placed
// between the stage VJPs, keeps the compiler from holding the slots in
// registers across them (which would bring the register pressure back); for
// ThetaBar (registers) it is a no-op.
struct LdsAcc {
  float* p;
  __device__ __forceinline__ void operator+=(float v) const { *p = *p + v; }
  __device__ __forceinline__ void operator-=(float v) const { *p = *p - v; }
};
struct LdsAccRow {
  float* p;
  __device__ __forceinline__ LdsAcc operator[](int i) const { return {p + i * kBlock}; }
};
struct ThetaBarLds {
  LdsAccRow ma, dl, dq;
  LdsAcc wmb, hz;
};
// slot k of a lane's column: ma 0-5, dl 6-11, dq 12-17, wmb 18, hz 19
__device__ __forceinline__ ThetaBarLds theta_bar_lds(float* col) {
#pragma unroll
  for (int k = 0; k < 20; ++k) col[k * kBlock] = 0.0f;
  return {{col}, {col + 6 * kBlock}, {col + 12 * kBlock}, {col + 18 * kBlock},
          {col + 19 * kBlock}};
}
template <class T>
__host__ __device__ __forceinline__ void theta_bar_fence(ThetaBar<T>&) {}
__device__ __forceinline__ void theta_bar_fence(ThetaBarLds&) { asm volatile("" ::: "memory"); }
template <class T>
__host__ __device__ __forceinline__ T theta_bar_get(const ThetaBar<T>& t, int k) {
  return k < 6 ? t.ma[k] : k < 12 ? t.dl[k - 6] : k < 18 ? t.dq[k - 12] : k == 18 ? t.wmb : t.hz;
}
__device__ __forceinline__ float theta_bar_get(const ThetaBarLds& t, int k) {
  return *(volatile float*)(t.ma.p + k * kBlock);
}

// dL/d(x, tau, theta) of xd = rhs_core(x, tau) given xdb = dL/dxd.
// Accumulates into xb (13 rows; the position rows receive nothing) and thb;
// writes taub.
template <class T, class TB>
__host__ __device__ __forceinline__ void rhs_core_vjp(const T* x, const EnvConstT<T>& P,
                                                      const T (&tau)[6], const T* xdb, T* xb,
                                                      T (&taub)[6], TB& thb) {
  const T qw = x[3], qx = x[4], qy = x[5], qz = x[6];
  const T u = x[7], v = x[8], w = x[9], p = x[10], q = x[11], r = x[12];
  // forward intermediates
  const T x2 = qx + qx, y2 = qy + qy, z2 = qz + qz;
  const T t0 = fma_t(y2, w, -z2 * v);
  const T t1 = fma_t(z2, u, -x2 * w);
  const T t2 = fma_t(x2, v, -y2 * u);
  const T k0 = fma_t(x2, qz, -y2 * qw);
  const T k1 = fma_t(y2, qz, x2 * qw);
  const T k2 = fma_t(-y2, qy, fma_t(-x2, qx, T(1)));
  const T au = fma_t(P.Muq, q, P.Muu * u), av = fma_t(P.Mvp, p, P.Mvv * v), aw = P.Mww * w;
  const T bp = fma_t(P.Mpp, p, P.Mvp * v), bq = fma_t(P.Mqq, q, P.Muq * u), br = P.Mrr * r;
  const T nu[6] = {u, v, w, p, q, r};
  T e[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) e[i] = fma_t(P.dq[i], abs_t(nu[i]), P.dl[i]);
  const T r0 = fma_t(-e[0], u, fma_t(P.wmb, k0, fma_t(-q, aw, fma_t(r, av, tau[0]))));
  const T r1 = fma_t(-e[1], v, fma_t(P.wmb, k1, fma_t(-r, au, fma_t(p, aw, tau[1]))));
  const T r2 = fma_t(-e[2], w, fma_t(P.wmb, k2, fma_t(-p, av, fma_t(q, au, tau[2]))));
  const T r3 = fma_t(-e[3], p, fma_t(-P.hz, k1,
               fma_t(r, bq, fma_t(-q, br, fma_t(w, av, fma_t(-v, aw, tau[3]))))));
  const T r4 = fma_t(-e[4], q, fma_t(P.hz, k0,
               fma_t(p, br, fma_t(-r, bp, fma_t(u, aw, fma_t(-w, au, tau[4]))))));
  const T r5 = fma_t(-e[5], r, fma_t(q, bp, fma_t(-p, bq, fma_t(v, au, fma_t(-u, av, tau[5])))));
  const T nud[6] = {fma_t(P.Iuq, r4, P.Iuu * r0), fma_t(P.Ivp, r3, P.Ivv * r1), P.Iww * r2,
                    fma_t(P.Ipp, r3, P.Ivp * r1), fma_t(P.Iqq, r4, P.Iuq * r0), P.Irr * r5};

  // nu' = M^-1 r:  rb = M^-1 nudb (M symmetric);  dM_ii gets -rb_i nud_i
  const T gu = xdb[7], gv = xdb[8], gw = xdb[9], gp = xdb[10], gq = xdb[11], gr = xdb[12];
  T rb[6];
  rb[0] = fma_t(P.Iuq, gq, P.Iuu * gu);
  rb[4] = fma_t(P.Iqq, gq, P.Iuq * gu);
  rb[1] = fma_t(P.Ivp, gp, P.Ivv * gv);
  rb[3] = fma_t(P.Ipp, gp, P.Ivp * gv);
  rb[2] = mul_nc(P.Iww, gw);
  rb[5] = mul_nc(P.Irr, gr);
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    thb.ma[i] -= rb[i] * nud[i];
    taub[i] = rb[i];
  }
  // residual rows
  T nub[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};   // u v w p q r
  T aub = T(0), avb = T(0), awb = T(0), bpb = T(0), bqb = T(0), brb = T(0);
  T k0b = T(0), k1b = T(0), k2b = T(0);
  T eb[6];
  // r0 = tau0 + r av - q aw + wmb k0 - e0 u
  nub[5] += av * rb[0]; avb += r * rb[0]; nub[4] -= aw * rb[0]; awb -= q * rb[0];
  k0b += P.wmb * rb[0]; thb.wmb += k0 * rb[0]; eb[0] = mul_nc(-u, rb[0]); nub[0] -= e[0] * rb[0];
  // r1 = tau1 + p aw - r au + wmb k1 - e1 v
  nub[3] += aw * rb[1]; awb += p * rb[1]; nub[5] -= au * rb[1]; aub -= r * rb[1];
  k1b += P.wmb * rb[1]; thb.wmb += k1 * rb[1]; eb[1] = mul_nc(-v, rb[1]); nub[1] -= e[1] * rb[1];
  // r2 = tau2 + q au - p av + wmb k2 - e2 w
  nub[4] += au * rb[2]; aub += q * rb[2]; nub[3] -= av * rb[2]; avb -= p * rb[2];
  k2b += P.wmb * rb[2]; thb.wmb += k2 * rb[2]; eb[2] = mul_nc(-w, rb[2]); nub[2] -= e[2] * rb[2];
  // r3 = tau3 - v aw + w av - q br + r bq - hz k1 - e3 p
  nub[1] -= aw * rb[3]; awb -= v * rb[3]; nub[2] += av * rb[3]; avb += w * rb[3];
  nub[4] -= br * rb[3]; brb -= q * rb[3]; nub[5] += bq * rb[3]; bqb += r * rb[3];
  k1b -= P.hz * rb[3]; thb.hz -= k1 * rb[3]; eb[3] = mul_nc(-p, rb[3]); nub[3] -= e[3] * rb[3];
  // r4 = tau4 - w au + u aw - r bp + p br + hz k0 - e4 q
  nub[2] -= au * rb[4]; aub -= w * rb[4]; nub[0] += aw * rb[4]; awb += u * rb[4];
  nub[5] -= bp * rb[4]; bpb -= r * rb[4]; nub[3] += br * rb[4]; brb += p * rb[4];
  k0b += P.hz * rb[4]; thb.hz += k0 * rb[4]; eb[4] = mul_nc(-q, rb[4]); nub[4] -= e[4] * rb[4];
  // r5 = tau5 - u av + v au - p bq + q bp - e5 r
  nub[0] -= av * rb[5]; avb -= u * rb[5]; nub[1] += au * rb[5]; aub += v * rb[5];
  nub[3] -= bq * rb[5]; bqb -= p * rb[5]; nub[4] += bp * rb[5]; bpb += q * rb[5];
  eb[5] = mul_nc(-r, rb[5]); nub[5] -= e[5] * rb[5];
  // e_i = d_L,i + d_Q,i |nu_i|   (d|x|/dx taken as +1 at 0)
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    thb.dl[i] += eb[i];
    thb.dq[i] += eb[i] * abs_t(nu[i]);
    nub[i] += (nu[i] < T(0) ? -P.dq[i] : P.dq[i]) * eb[i];
  }
  // [a; b] = M nu
  nub[0] += P.Muu * aub; nub[4] += P.Muq * aub; thb.ma[0] += u * aub;
  nub[1] += P.Mvv * avb; nub[3] += P.Mvp * avb; thb.ma[1] += v * avb;
  nub[2] += P.Mww * awb; thb.ma[2] += w * awb;
  nub[1] += P.Mvp * bpb; nub[3] += P.Mpp * bpb; thb.ma[3] += p * bpb;
  nub[0] += P.Muq * bqb; nub[4] += P.Mqq * bqb; thb.ma[4] += q * bqb;
  nub[5] += P.Mrr * brb; thb.ma[5] += r * brb;
  // quaternion rows (xd[3..6] = q (x) (0, w))
  const T g0 = xdb[0], g1 = xdb[1], g2 = xdb[2];
  const T g3 = xdb[3], g4 = xdb[4], g5 = xdb[5], g6 = xdb[6];
  T qwb = T(0), qxb = T(0), qyb = T(0), qzb = T(0);
  qxb -= p * g3; nub[3] -= qx * g3; qyb -= q * g3; nub[4] -= qy * g3; qzb -= r * g3;
  nub[5] -= qz * g3;
  qwb += p * g4; nub[3] += qw * g4; qyb += r * g4; nub[5] += qy * g4; qzb -= q * g4;
  nub[4] -= qz * g4;
  qwb += q * g5; nub[4] += qw * g5; qzb += p * g5; nub[3] += qz * g5; qxb -= r * g5;
  nub[5] -= qx * g5;
  qwb += r * g6; nub[5] += qw * g6; qxb += q * g6; nub[4] += qx * g6; qyb -= p * g6;
  nub[3] -= qy * g6;
  // k = R^T e3
  T x2b = T(0), y2b = T(0), z2b = T(0);
  x2b += qz * k0b; qzb += x2 * k0b; y2b -= qw * k0b; qwb -= y2 * k0b;
  y2b += qz * k1b; qzb += y2 * k1b; x2b += qw * k1b; qwb += x2 * k1b;
  x2b -= qx * k2b; qxb -= x2 * k2b; y2b -= qy * k2b; qyb -= y2 * k2b;
  // p' = v + qw t + q_v x t,  t = 2 q_v x v
  T t0b = T(0), t1b = T(0), t2b = T(0);
  nub[0] += g0; qwb += t0 * g0; t0b += qw * g0; qyb += t2 * g0; t2b += qy * g0;
  qzb -= t1 * g0; t1b -= qz * g0;
  nub[1] += g1; qwb += t1 * g1; t1b += qw * g1; qzb += t0 * g1; t0b += qz * g1;
  qxb -= t2 * g1; t2b -= qx * g1;
  nub[2] += g2; qwb += t2 * g2; t2b += qw * g2; qxb += t1 * g2; t1b += qx * g2;
  qyb -= t0 * g2; t0b -= qy * g2;
  y2b += w * t0b; nub[2] += y2 * t0b; z2b -= v * t0b; nub[1] -= z2 * t0b;
  z2b += u * t1b; nub[0] += z2 * t1b; x2b -= w * t1b; nub[2] -= x2 * t1b;
  x2b += v * t2b; nub[1] += x2 * t2b; y2b -= u * t2b; nub[0] -= y2 * t2b;
  qxb += T(2) * x2b;
  qyb += T(2) * y2b;
  qzb += T(2) * z2b;
  xb[3] += qwb;
  xb[4] += qxb;
  xb[5] += qyb;
  xb[6] += qzb;
#pragma unroll
  for (int i = 0; i < 6; ++i) xb[7 + i] += nub[i];
}

// Reverse of rk4_substep: y is the sub-step input (D rows), lam holds dL/d(output)
// on entry and dL/dy on exit; dL/d f_cmd and dL/d (B f_cmd) accumulate into fcb and
// gcb, parameter adjoints into thb.
template <int N, bool LAG, class T, class TB>
__host__ __device__ __forceinline__ void rk4_substep_vjp(const T* y, const EnvConstT<T>& P,
                                                         const ClassConst& cc,
                                                         const T (&fcmd)[N], const T (&gcmd)[6],
                                                         T dt, T* lam, T (&fcb)[N], T (&gcb)[6],
                                                         TB& thb) {
  const T h2 = T(0.5) * dt, h6 = dt * (T(1) / T(6));
  auto fac = [](int i, T f) { return (i >= 3 && i < 7) ? T(0.5) * f : f; };
  T df[N], dg[6], tau1[6], tau2[6], tau3[6], tau4[6];
  if constexpr (LAG) {
#pragma unroll
    for (int i = 0; i < N; ++i) df[i] = y[13 + i] - fcmd[i];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      T s = mul_nc(T(cc.B[k][0]), df[0]);
#pragma unroll
      for (int i = 1; i < N; ++i) s = fma_t(T(cc.B[k][i]), df[i], s);
      dg[k] = s;
      tau1[k] = gcmd[k] + s;
      tau2[k] = fma_t(T(cc.sigma2), s, gcmd[k]);
      tau3[k] = fma_t(T(cc.sigma3), s, gcmd[k]);
      tau4[k] = fma_t(T(cc.sigma4), s, gcmd[k]);
    }
  } else {
#pragma unroll
    for (int k = 0; k < 6; ++k) tau1[k] = tau2[k] = tau3[k] = tau4[k] = gcmd[k];
  }
  // forward recomputation of the stage inputs and of the pre-normalisation quaternion
  T k[13], acc[13], X2[13], X3[13], X4[13];
  rhs_core(y, k, P, tau1);
#pragma unroll
  for (int i = 0; i < 13; ++i) {
    acc[i] = k[i];
    X2[i] = fma_t(fac(i, h2), k[i], y[i]);
  }
  rhs_core(X2, k, P, tau2);
#pragma unroll
  for (int i = 0; i < 13; ++i) {
    acc[i] = fma_t(T(2), k[i], acc[i]);
    X3[i] = fma_t(fac(i, h2), k[i], y[i]);
  }
  rhs_core(X3, k, P, tau3);
#pragma unroll
  for (int i = 0; i < 13; ++i) {
    acc[i] = fma_t(T(2), k[i], acc[i]);
    X4[i] = fma_t(fac(i, dt), k[i], y[i]);
  }
  rhs_core(X4, k, P, tau4);
  T qt[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) qt[i] = fma_t(fac(3 + i, h6), acc[3 + i] + k[3 + i], y[3 + i]);

  // renormalisation q = qt / |qt|:  dqt = (lam_q - q (q . lam_q)) / |qt|
  const T n2 = qt[0] * qt[0] + qt[1] * qt[1] + qt[2] * qt[2] + qt[3] * qt[3];
  const T inv = rsqrt_t(n2);
  T qo[4], dot = T(0);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    qo[i] = qt[i] * inv;
    dot += qo[i] * lam[3 + i];
  }
  T zb[13];
#pragma unroll
  for (int i = 0; i < 13; ++i) zb[i] = lam[i];
#pragma unroll
  for (int i = 0; i < 4; ++i) zb[3 + i] = mul_nc(lam[3 + i] - qo[i] * dot, inv);

  // combination z' = y + fac(h6) (k1 + 2 k2 + 2 k3 + k4), then the stages in reverse
  T yb[13], kb[13], Xb[13], tb1[6], tb2[6], tb3[6], tb4[6];
#pragma unroll
  for (int i = 0; i < 13; ++i) {
    yb[i] = zb[i];
    kb[i] = mul_nc(fac(i, h6), zb[i]);
    Xb[i] = T(0);
  }
  theta_bar_fence(thb);
  rhs_core_vjp(X4, P, tau4, kb, Xb, tb4, thb);          // X4 = y + fac(dt) k3
#pragma unroll
  for (int i = 0; i < 13; ++i) {
    yb[i] += Xb[i];
    kb[i] = fma_t(fac(i, dt), Xb[i], T(2) * fac(i, h6) * zb[i]);
    Xb[i] = T(0);
  }
  theta_bar_fence(thb);
  rhs_core_vjp(X3, P, tau3, kb, Xb, tb3, thb);          // X3 = y + fac(h2) k2
#pragma unroll
  for (int i = 0; i < 13; ++i) {
    yb[i] += Xb[i];
    kb[i] = fma_t(fac(i, h2), Xb[i], T(2) * fac(i, h6) * zb[i]);
    Xb[i] = T(0);
  }
  theta_bar_fence(thb);
  rhs_core_vjp(X2, P, tau2, kb, Xb, tb2, thb);          // X2 = y + fac(h2) k1
#pragma unroll
  for (int i = 0; i < 13; ++i) {
    yb[i] += Xb[i];
    kb[i] = fma_t(fac(i, h2), Xb[i], fac(i, h6) * zb[i]);
    Xb[i] = T(0);
  }
  theta_bar_fence(thb);
  rhs_core_vjp(y, P, tau1, kb, Xb, tb1, thb);           // X1 = y
#pragma unroll
  for (int i = 0; i < 13; ++i) lam[i] = yb[i] + Xb[i];

  // stage wrenches tau_i = B f_cmd + sigma_i B (f - f_cmd) and f' = f_cmd + rho (f - f_cmd)
  if constexpr (LAG) {
    T dgb[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      gcb[j] += (tb1[j] + tb2[j]) + (tb3[j] + tb4[j]);
      dgb[j] = tb1[j] + T(cc.sigma2) * tb2[j] + T(cc.sigma3) * tb3[j] + T(cc.sigma4) * tb4[j];
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const T fob = lam[13 + i];
      T dfb = T(cc.rho) * fob;
#pragma unroll
      for (int j = 0; j < 6; ++j) dfb = fma_t(T(cc.B[j][i]), dgb[j], dfb);
      fcb[i] += fob - dfb;
      lam[13 + i] = dfb;
    }
    (void)dg;
  } else {
#pragma unroll
    for (int j = 0; j < 6; ++j) gcb[j] += (tb1[j] + tb2[j]) + (tb3[j] + tb4[j]);
  }
}

// dL/d throttle from dL/d f_cmd (and dL/d (B f_cmd)), through the clamp and the thrust map.
template <int N, class T>
__host__ __device__ __forceinline__ void throttle_vjp(const ClassConst& cc, const T (&a)[N],
                                                      T (&fcb)[N], const T (&gcb)[6],
                                                      T (&ab)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T s = fcb[i];
#pragma unroll
    for (int j = 0; j < 6; ++j) s = fma_t(T(cc.B[j][i]), gcb[j], s);
    const bool inside = !(a[i] > T(1)) && !(a[i] < T(-1));
    const T slope = cc.thr_map ? T(2) * T(cc.f_max) * abs_t(a[i]) : T(cc.f_max);
    ab[i] = inside ? s * slope : T(0);
  }
}

// ---- the backward of one env over a checkpointed rollout -------------------
// (kernels_adjoint.hip launches these, one lane per env; host and device code,
// so that the same source also runs on the CPU in tests)

template <int N>
__host__ __device__ __forceinline__ void load_command(const ClassConst& cc, const AdjArgs& a, int t,
                                             int64_t c, float (&act)[N], float (&fcmd)[N],
                                             float (&gcmd)[6]) {
  const float* af = a.actions + (int64_t)t * a.n_max * a.E + c;
#pragma unroll
  for (int i = 0; i < N; ++i) act[i] = af[i * a.E];
  thrust_command<N>(cc, act, fcmd);
  command_wrench<N>(cc, fcmd, gcmd);
}

// Recomputes the sub-step inputs of control steps [t0, t1) from the state x
// at t0 into segbuf rows (t - base) * S + s.  The forward sets the lag states
// to their end-of-control-step value at the start; the sub-step inputs the VJP
// linearises about carry the lag states of each sub-step, f_cmd + rho^s
// (f - f_cmd), kept here in fs.
// Used by k_adj_recompute only: the backward keeps its own copy of this loop
// (see adj_bwd_env).
template <int N, bool LAG>
__host__ __device__ __forceinline__ void recompute_segment(const AdjArgs& a, const ClassConst& cc,
                                                  const EnvConst& P, const HalfInvT<float>& A,
                                                  const StepConstT<float>& sc,
                                                  float (&x)[Dims<N, LAG>::D], int t0, int t1,
                                                  int base, int64_t j, int64_t c) {
  constexpr int D = Dims<N, LAG>::D;
  const int S = a.substeps;
  for (int t = t0; t < t1; ++t) {
    float act[N], fcmd[N], gcmd[6], dg[6], fs[LAG ? N : 1];
    load_command<N>(cc, a, t, c, act, fcmd, gcmd);
    if constexpr (LAG) {
#pragma unroll
      for (int i = 0; i < N; ++i) fs[i] = x[13 + i];
    }
    begin_control_step<N, LAG>(cc, x, fcmd, dg, cc.rho_s);
    float m[6];
    momentum(P, x + 7, m);
    for (int s = 0; s < S; ++s) {
      float* sb = a.segbuf + (int64_t)((t - base) * S + s) * D * a.Ep + j;
#pragma unroll
      for (int i = 0; i < 13; ++i) sb[i * a.Ep] = x[i];
      if constexpr (LAG) {
#pragma unroll
        for (int i = 0; i < N; ++i) {
          sb[(13 + i) * a.Ep] = fs[i];
          fs[i] = fma_t(sc.rho, fs[i] - fcmd[i], fcmd[i]);
        }
      }
      rk4_substep<N, LAG>(x, m, P, A, gcmd, dg, sc);
    }
  }
}

// WHOLE: the sub-step inputs of the whole rollout are already in segbuf
// (k_adj_recompute); otherwise each segment is recomputed here, into a
// segment-sized segbuf, just before its sweep.  The recomputation loop is
// written out here rather than calling recompute_segment: with that call
// inlined, the one-wave 8-thruster lag instantiation (256 VGPRs + AGPRs)
// returned gradients 5e-2 away from the oracle's although the source was
// equivalent, and out of line the call's register saves made the kernel 2-3x
// slower; this loop, unchanged, matches the oracle to 5e-7.
//
// adj_bwd_env is the backward of one env: internal column j, caller column c,
// its constants P, the step factors sc and the pre-scaled inverse A.  Host and
// device code, so that the same source also runs on the CPU (tests); the
// kernel k_adj_bwd below loads the env's constants and inlines it.
// PREFETCH: the next sub-step's input and the next control step's dL/d traj
// and throttles are loaded one step ahead, so that their latency hides
// behind the current sub-step's VJP (a launch of one wave per SIMD has no
// other wave to hide it behind); it costs 2 D + N registers, which the
// two-wave build cannot spare.
// TRAJ (with WHOLE): one sub-step per control step, each step's input read
// from the caller's trajectory instead of the recomputation buffer.
// TB: ThetaBar<float> (registers) or ThetaBarLds (LDS), zeroed by the caller;
// the parameter adjoints accumulate into it and are written out at the end.
template <int N, bool LAG, bool WHOLE, bool PREFETCH = false, bool TRAJ = false,
          class TB = ThetaBar<float>>
__host__ __device__ __forceinline__ void adj_bwd_env(const AdjArgs& a, const ClassConst& cc,
                                                     const EnvConst& P,
                                                     const StepConstT<float>& sc,
                                                     const HalfInvT<float>& A, int64_t j,
                                                     int64_t c, TB thb) {
  constexpr int D = Dims<N, LAG>::D;
  const int K = a.ckpt_every, S = a.substeps;
  const int nseg = (a.T + K - 1) / K;
  static_assert(WHOLE || !TRAJ, "trajectory inputs replace the whole-rollout buffer");
  // the input of sub-step s of control step t: from the recomputation buffer,
  // or (TRAJ: one sub-step per control step) from the caller's trajectory row
  // of the step before, the first checkpoint for t = 0
  auto load_input = [&](int t, int s, int base, float (&y)[D]) {
    if constexpr (TRAJ) {
      (void)s;
      (void)base;
      const float* p = t == 0 ? a.ckpt + c : a.traj + (int64_t)(t - 1) * a.D * a.E + c;
#pragma unroll
      for (int i = 0; i < D; ++i) y[i] = p[i * a.E];
    } else {
      const float* sb = a.segbuf + (int64_t)((t - base) * S + s) * D * a.Ep + j;
#pragma unroll
      for (int i = 0; i < D; ++i) y[i] = sb[i * a.Ep];
    }
  };
  float lam[D];
#pragma unroll
  for (int i = 0; i < D; ++i) lam[i] = 0.0f;
  for (int seg = nseg - 1; seg >= 0; --seg) {
    const int t0 = seg * K, t1 = min(a.T, t0 + K);
    const int base = WHOLE ? 0 : t0;   // segbuf row of control step t: (t - base) * S
    if constexpr (!WHOLE) {
      // recompute this segment's sub-step inputs from its checkpoint
      float x[D];
      const float* ck = a.ckpt + (int64_t)seg * a.D * a.E + c;
#pragma unroll
      for (int i = 0; i < D; ++i) x[i] = ck[i * a.E];
      // (the forward sets the lag states to their end-of-control-step value at
      // the start; the sub-step inputs the VJP linearises about carry the lag
      // states of each sub-step, f_cmd + rho^s (f - f_cmd), kept here in fs)
      for (int t = t0; t < t1; ++t) {
        float act[N], fcmd[N], gcmd[6], dg[6], fs[LAG ? N : 1];
        load_command<N>(cc, a, t, c, act, fcmd, gcmd);
        if constexpr (LAG) {
#pragma unroll
          for (int i = 0; i < N; ++i) fs[i] = x[13 + i];
        }
        begin_control_step<N, LAG>(cc, x, fcmd, dg, cc.rho_s);
        float m[6];
        momentum(P, x + 7, m);
        for (int s = 0; s < S; ++s) {
          float* sb = a.segbuf + (int64_t)((t - t0) * S + s) * D * a.Ep + j;
#pragma unroll
          for (int i = 0; i < 13; ++i) sb[i * a.Ep] = x[i];
          if constexpr (LAG) {
#pragma unroll
            for (int i = 0; i < N; ++i) {
              sb[(13 + i) * a.Ep] = fs[i];
              fs[i] = fma_t(sc.rho, fs[i] - fcmd[i], fcmd[i]);
            }
          }
          rk4_substep<N, LAG>(x, m, P, A, gcmd, dg, sc);
        }
      }
    }
    // reverse sweep over the segment
    if constexpr (PREFETCH) {
      float y_n[D], gt_n[D], act_n[N];
      {
        load_input(t1 - 1, S - 1, base, y_n);
        const float* gt = a.gtraj + (int64_t)(t1 - 1) * a.D * a.E + c;
#pragma unroll
        for (int i = 0; i < D; ++i) gt_n[i] = gt[i * a.E];
        const float* af = a.actions + (int64_t)(t1 - 1) * a.n_max * a.E + c;
#pragma unroll
        for (int i = 0; i < N; ++i) act_n[i] = af[i * a.E];
      }
      for (int t = t1 - 1; t >= t0; --t) {
        float act[N], fcmd[N], gcmd[6], fcb[N], gcb[6], ab[N];
#pragma unroll
        for (int i = 0; i < D; ++i) lam[i] += gt_n[i];
#pragma unroll
        for (int i = 0; i < N; ++i) act[i] = act_n[i];
        if (t > t0) {
          const float* gt = a.gtraj + (int64_t)(t - 1) * a.D * a.E + c;
#pragma unroll
          for (int i = 0; i < D; ++i) gt_n[i] = gt[i * a.E];
          const float* af = a.actions + (int64_t)(t - 1) * a.n_max * a.E + c;
#pragma unroll
          for (int i = 0; i < N; ++i) act_n[i] = af[i * a.E];
        }
        thrust_command<N>(cc, act, fcmd);
        command_wrench<N>(cc, fcmd, gcmd);
#pragma unroll
        for (int i = 0; i < N; ++i) fcb[i] = 0.0f;
#pragma unroll
        for (int k = 0; k < 6; ++k) gcb[k] = 0.0f;
        for (int s = S - 1; s >= 0; --s) {
          float y[D];
#pragma unroll
          for (int i = 0; i < D; ++i) y[i] = y_n[i];
          if (s > 0)
            load_input(t, s - 1, base, y_n);
          else if (t > t0)
            load_input(t - 1, S - 1, base, y_n);
          rk4_substep_vjp<N, LAG>(y, P, cc, fcmd, gcmd, a.dt, lam, fcb, gcb, thb);
        }
        throttle_vjp<N>(cc, act, fcb, gcb, ab);
        float* ga = a.gact + (int64_t)t * a.n_max * a.E + c;
#pragma unroll
        for (int i = 0; i < N; ++i) ga[i * a.E] = ab[i];
        for (int i = N; i < a.n_max; ++i) ga[i * a.E] = 0.0f;
      }
    } else {
      for (int t = t1 - 1; t >= t0; --t) {
        const float* gt = a.gtraj + (int64_t)t * a.D * a.E + c;
#pragma unroll
        for (int i = 0; i < D; ++i) lam[i] += gt[i * a.E];
        float act[N], fcmd[N], gcmd[6], fcb[N], gcb[6], ab[N];
        load_command<N>(cc, a, t, c, act, fcmd, gcmd);
#pragma unroll
        for (int i = 0; i < N; ++i) fcb[i] = 0.0f;
#pragma unroll
        for (int k = 0; k < 6; ++k) gcb[k] = 0.0f;
        if constexpr (TRAJ) {   // one sub-step per control step
          float y[D];
          load_input(t, 0, base, y);
          rk4_substep_vjp<N, LAG>(y, P, cc, fcmd, gcmd, a.dt, lam, fcb, gcb, thb);
        } else {
          for (int s = S - 1; s >= 0; --s) {
            float y[D];
            load_input(t, s, base, y);
            rk4_substep_vjp<N, LAG>(y, P, cc, fcmd, gcmd, a.dt, lam, fcb, gcb, thb);
          }
        }
        throttle_vjp<N>(cc, act, fcb, gcb, ab);
        float* ga = a.gact + (int64_t)t * a.n_max * a.E + c;
#pragma unroll
        for (int i = 0; i < N; ++i) ga[i * a.E] = ab[i];
        for (int i = N; i < a.n_max; ++i) ga[i * a.E] = 0.0f;
      }
    }
  }
  // theta = (M_A(6), D_L(6), D_Q(6), B);  W - B and h_z = W z_g - B z_b carry B
#pragma unroll
  for (int k = 0; k < 18; ++k) a.gtheta[k * a.E + c] = theta_bar_get(thb, k);
  a.gtheta[18 * a.E + c] = -theta_bar_get(thb, 18) - a.zb * theta_bar_get(thb, 19);
  if (a.gx0) {
#pragma unroll
    for (int i = 0; i < D; ++i) a.gx0[i * a.E + c] = lam[i];
    for (int i = D; i < a.D; ++i) a.gx0[i * a.E + c] = 0.0f;
  }
}

}  // namespace mg
