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
#include "page_pool.h"

namespace mg {

// Scalar helpers; the double versions serve host-side checks of the kernel math.
__host__ __device__ inline float fma_t(float a, float b, float c) { return fmaf(a, b, c); }
__host__ __device__ inline double fma_t(double a, double b, double c) { return fma(a, b, c); }

// A product never fused into an FMA with the sum it feeds.  Where a product
// has several uses and one of them is a sum, whether the compiler contracts
// that sum depends on the rest of the kernel, so two kernels built from the
// same code (the step, the adjoint's forward and recomputation, the one-wave,
// two-wave and trajectory-reading sweeps) could round it differently.  The
// products of that kind go through mul_nc, which keeps results bitwise equal
// across kernels.
template <class T>
__host__ __device__ __forceinline__ T mul_nc(T a, T b) {
#pragma clang fp contract(off)
  return a * b;
}

__host__ __device__ inline float abs_t(float a) { return fabsf(a); }
__host__ __device__ inline double abs_t(double a) { return fabs(a); }
// Used only for 1/|q| with |q|^2 close to 1 (never denormal): the hardware
// reciprocal square root (v_rsq_f32, 1 ulp) without the denormal rescaling
// rsqrtf wraps around it, which gives the same value for normal inputs.
__device__ inline float rsqrt_t(float a) { return __builtin_amdgcn_rsqf(a); }
// host overload (CPU checks of the FP32 code): correctly rounded sqrt, then divide
__host__ inline float rsqrt_t(float a) { return 1.0f / sqrtf(a); }
__host__ __device__ inline double rsqrt_t(double a) { return 1.0 / sqrt(a); }

// Per-env constants held in registers for the whole launch.
template <class T>
struct EnvConstT {
  T Muu, Mvv, Mww, Mpp, Mqq, Mrr, Muq, Mvp;
  T Iuu, Ivv, Iww, Ipp, Iqq, Irr, Iuq, Ivp;
  T dl[6], dq[6];
  T wmb, hz;
};
using EnvConst = EnvConstT<float>;

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

// Uniform per-launch factors of the RK4 sub-step.  On gfx950 a VALU
// instruction that reads a scalar register does not dual-issue, so the kernels
// copy these into vector registers once (to_vgpr) and the sub-step's FMAs read
// only vector registers.
template <class T>
struct StepConstT {
  T h2, h2q, dt, dtq, h6, h6q;   // stage / combination factors; *q: quaternion rows (x 1/2)
  T two, third;
  T s2, s3, s4, rho;             // closed-form lag stage factors (ClassConst)
};

__device__ __forceinline__ float to_vgpr(float x) {
  float r;
  asm("v_mov_b32 %0, %1" : "=v"(r) : "s"(x));
  return r;
}

__device__ __forceinline__ StepConstT<float> make_step_const(const ClassConst& cc, float dt) {
  StepConstT<float> k;
  const float h2 = 0.5f * dt, h6 = dt * (1.0f / 6.0f);
  k.h2 = to_vgpr(h2);
  k.h2q = to_vgpr(0.5f * h2);
  k.dt = to_vgpr(dt);
  k.dtq = to_vgpr(0.5f * dt);
  k.h6 = to_vgpr(h6);
  k.h6q = to_vgpr(0.5f * h6);
  k.two = to_vgpr(2.0f);
  k.third = to_vgpr(1.0f / 3.0f);
  k.s2 = to_vgpr(cc.sigma2);
  k.s3 = to_vgpr(cc.sigma3);
  k.s4 = to_vgpr(cc.sigma4);
  k.rho = to_vgpr(cc.rho);
  return k;
}

// Host-side (double) version for checks of the kernel math.
inline StepConstT<double> make_step_const_host(const ClassConst& cc, double dt) {
  StepConstT<double> k;
  const double h2 = 0.5 * dt, h6 = dt * (1.0 / 6.0);
  k.h2 = h2; k.h2q = 0.5 * h2; k.dt = dt; k.dtq = 0.5 * dt; k.h6 = h6; k.h6q = 0.5 * h6;
  k.two = 2.0;
  k.third = 1.0 / 3.0;
  k.s2 = cc.sigma2; k.s3 = cc.sigma3; k.s4 = cc.sigma4; k.rho = cc.rho;
  return k;
}

// Per-env factorisation done once at reset: M = M_RB + M_A for diagonal I_g
// and M_A with r_g = (0,0,z_g) couples only (u,q) and (v,p), so M^-1 is two
// 2x2 inverses and two reciprocals; formed in FP64 from the parameters
// prm = (m, I(3), M_A(6), D_L(6), D_Q(6), B) and rounded once.  A mass matrix
// that is not positive definite yields NaN constants.
__device__ __forceinline__ void derive_constants(const double (&prm)[kNumParams], double zg,
                                                 double zb, float (&out)[kNumDerived]) {
  const double m = prm[0];
  const double Muu = m + prm[4], Mvv = m + prm[5], Mww = m + prm[6];
  const double mzz = mul_nc(mul_nc(m, zg), zg);   // m z_g^2 (two sums use it)
  const double Mpp = prm[1] + mzz + prm[7];
  const double Mqq = prm[2] + mzz + prm[8];
  const double Mrr = prm[3] + prm[9];
  const double Muq = m * zg, Mvp = -m * zg;
  const double det_uq = Muu * Mqq - Muq * Muq, det_vp = Mvv * Mpp - Mvp * Mvp;
  const bool spd = Muu > 0.0 && Mvv > 0.0 && Mww > 0.0 && Mrr > 0.0 && det_uq > 0.0 &&
                   det_vp > 0.0;
  double dv[kNumDerived];
  dv[kMuu] = Muu; dv[kMvv] = Mvv; dv[kMww] = Mww; dv[kMpp] = Mpp; dv[kMqq] = Mqq;
  dv[kMrr] = Mrr; dv[kMuq] = Muq; dv[kMvp] = Mvp;
  dv[kIuu] = Mqq / det_uq; dv[kIqq] = Muu / det_uq; dv[kIuq] = -Muq / det_uq;
  dv[kIvv] = Mpp / det_vp; dv[kIpp] = Mvv / det_vp; dv[kIvp] = -Mvp / det_vp;
  dv[kIww] = 1.0 / Mww; dv[kIrr] = 1.0 / Mrr;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    dv[kDL + i] = prm[10 + i];
    dv[kDQ + i] = prm[16 + i];
  }
  const double W = mul_nc(m, kG0), B = prm[22];
  dv[kWmB] = W - B;
  dv[kHz] = W * zg - B * zb;
#pragma unroll
  for (int i = 0; i < kNumDerived; ++i) out[i] = spd ? (float)dv[i] : __builtin_nanf("");
}

// One env's parameters: the class nominal values times the multipliers
// in[i * stride] (absolute values if `absolute`; nominal if in is NULL),
// each rounded once to FP32 and stored, and the factorisation derived from
// the stored FP32 values (so a sim restored from its parameters reproduces
// the original bitwise).
// Returns false when the mass matrix is not positive definite (or a parameter
// is not finite): the derived constants are then NaN.
__device__ __forceinline__ bool set_env_params(const ClassNominal& nom, const float* in,
                                               int64_t stride, bool absolute, float* params,
                                               float* derived, int64_t Ep, int64_t j) {
  double prm[kNumParams];
#pragma unroll
  for (int i = 0; i < kNumParams; ++i) {
    double pi = nom.p[i];
    if (in) {
      const double v = in[i * stride];
      pi = absolute ? v : pi * v;
    }
    const float pf = (float)pi;
    prm[i] = (double)pf;
    params[i * Ep + j] = pf;
  }
  float dvf[kNumDerived];
  derive_constants(prm, nom.zg, nom.zb, dvf);
  bool ok = true;
#pragma unroll
  for (int i = 0; i < kNumDerived; ++i) {
    derived[i * Ep + j] = dvf[i];
    ok = ok && isfinite(dvf[i]);
  }
  return ok;
}

// Row-plus-lane addressing for the step kernel.  A row pointer that is the
// same for the whole wave is pinned in scalar registers (the empty asm keeps
// the compiler from folding the lane's offset into it), and the lane's byte
// offset (below 4 GiB: at most 2^30 envs) is added as a 32-bit vector offset,
// so each load or store is one global_load / global_store with an SGPR base
// and no 64-bit index arithmetic per access.  Only wave-uniform pointers may
// be passed as `row`.
template <class T>
__device__ __forceinline__ T* pin_sgpr(T* p) {
  uint64_t v = reinterpret_cast<uint64_t>(p);
  asm volatile("" : "+s"(v));
  return reinterpret_cast<T*>(v);
}
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T& lane_elem(T* row, uint32_t off) {
  using G = __attribute__((address_space(1))) char;
  G* b = (G*)(pin_sgpr(row));
  return *(__attribute__((address_space(1))) T*)(b + off);
}
template <class T>
__device__ __forceinline__ const __attribute__((address_space(1))) T& lane_elem(const T* row,
                                                                                uint32_t off) {
  using G = const __attribute__((address_space(1))) char;
  G* b = (G*)(pin_sgpr(row));
  return *(const __attribute__((address_space(1))) T*)(b + off);
}

__device__ __forceinline__ EnvConst load_env_const_off(const float* __restrict__ der, int64_t Ep,
                                                       uint32_t off) {
  EnvConst P;
  P.Muu = lane_elem(der + kMuu * Ep, off); P.Mvv = lane_elem(der + kMvv * Ep, off);
  P.Mww = lane_elem(der + kMww * Ep, off); P.Mpp = lane_elem(der + kMpp * Ep, off);
  P.Mqq = lane_elem(der + kMqq * Ep, off); P.Mrr = lane_elem(der + kMrr * Ep, off);
  P.Muq = lane_elem(der + kMuq * Ep, off); P.Mvp = lane_elem(der + kMvp * Ep, off);
  P.Iuu = lane_elem(der + kIuu * Ep, off); P.Ivv = lane_elem(der + kIvv * Ep, off);
  P.Iww = lane_elem(der + kIww * Ep, off); P.Ipp = lane_elem(der + kIpp * Ep, off);
  P.Iqq = lane_elem(der + kIqq * Ep, off); P.Irr = lane_elem(der + kIrr * Ep, off);
  P.Iuq = lane_elem(der + kIuq * Ep, off); P.Ivp = lane_elem(der + kIvp * Ep, off);
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    P.dl[i] = lane_elem(der + (kDL + i) * Ep, off);
    P.dq[i] = lane_elem(der + (kDQ + i) * Ep, off);
  }
  P.wmb = lane_elem(der + kWmB * Ep, off);
  P.hz = lane_elem(der + kHz * Ep, off);
  return P;
}

template <int N, bool LAG>
struct Dims {
  static constexpr int D = 13 + (LAG ? N : 0);
};

// Commanded thrust from a throttle frame (Eq. (3)): clamp to [-1,1], then
// f_max a (linear) or f_max a|a| (quadratic).
template <int N, class T>
__host__ __device__ __forceinline__ void thrust_command(const ClassConst& cc, const T (&a)[N],
                                                        T (&fcmd)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    // fminf/fmaxf would turn a NaN throttle into a number; keep NaN flowing
    T ai = a[i] > T(1) ? T(1) : (a[i] < T(-1) ? T(-1) : a[i]);
    fcmd[i] = cc.thr_map ? T(cc.f_max) * ai * abs_t(ai) : T(cc.f_max) * ai;
  }
}

// Wrench of the commanded thrust, B f_cmd (once per control step).
template <int N, class T>
__host__ __device__ __forceinline__ void command_wrench(const ClassConst& cc, const T (&fcmd)[N],
                                                        T (&gcmd)[6]) {
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    T s = mul_nc(T(cc.B[k][0]), fcmd[0]);
#pragma unroll
    for (int i = 1; i < N; ++i) s = fma_t(T(cc.B[k][i]), fcmd[i], s);
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
// The momentum [a; b] = M nu of the structured M, ordered (u, v, w, p, q, r).
template <class T>
__host__ __device__ __forceinline__ void momentum(const EnvConstT<T>& P, const T* nu,
                                                  T (&mom)[6]) {
  const T u = nu[0], v = nu[1], w = nu[2], p = nu[3], q = nu[4], r = nu[5];
  mom[0] = fma_t(P.Muq, q, P.Muu * u);
  mom[1] = fma_t(P.Mvp, p, P.Mvv * v);
  mom[2] = P.Mww * w;
  mom[3] = fma_t(P.Mpp, p, P.Mvp * v);
  mom[4] = fma_t(P.Mqq, q, P.Muq * u);
  mom[5] = P.Mrr * r;
}

// rhs_residual_m writes the kinematic rows xd[0..6] and the residual
// r = tau - C nu - D nu - g given the momentum mom = M nu of the state x;
// rhs_residual forms mom itself; rhs_core applies M^-1 to the residual.  xd
// may not alias x.
template <class T>
__host__ __device__ __forceinline__ void rhs_residual_m(const T* x, const T (&mom)[6], T* xd,
                                                        T (&res)[6], const EnvConstT<T>& P,
                                                        const T (&tau)[6]) {
  const T qw = x[3], qx = x[4], qy = x[5], qz = x[6];
  const T u = x[7], v = x[8], w = x[9], p = x[10], q = x[11], r = x[12];

  // kinematics
  const T x2 = qx + qx, y2 = qy + qy, z2 = qz + qz;
  const T t0 = fma_t(y2, w, -z2 * v);
  const T t1 = fma_t(z2, u, -x2 * w);
  const T t2 = fma_t(x2, v, -y2 * u);
  xd[0] = fma_t(-qz, t1, fma_t(qy, t2, fma_t(qw, t0, u)));
  xd[1] = fma_t(-qx, t2, fma_t(qz, t0, fma_t(qw, t1, v)));
  xd[2] = fma_t(-qy, t0, fma_t(qx, t1, fma_t(qw, t2, w)));
  xd[3] = -fma_t(qx, p, fma_t(qy, q, qz * r));
  xd[4] = fma_t(-qz, q, fma_t(qy, r, qw * p));
  xd[5] = fma_t(-qx, r, fma_t(qz, p, qw * q));
  xd[6] = fma_t(-qy, p, fma_t(qx, q, qw * r));
  // k = R^T e3, the third row of R(q)
  const T k0 = fma_t(x2, qz, -y2 * qw);
  const T k1 = fma_t(y2, qz, x2 * qw);
  const T k2 = fma_t(-y2, qy, fma_t(-x2, qx, T(1)));

  const T au = mom[0], av = mom[1], aw = mom[2], bp = mom[3], bq = mom[4], br = mom[5];
  // damping coefficients d_L + d_Q |nu|
  const T e0 = fma_t(P.dq[0], abs_t(u), P.dl[0]);
  const T e1 = fma_t(P.dq[1], abs_t(v), P.dl[1]);
  const T e2 = fma_t(P.dq[2], abs_t(w), P.dl[2]);
  const T e3 = fma_t(P.dq[3], abs_t(p), P.dl[3]);
  const T e4 = fma_t(P.dq[4], abs_t(q), P.dl[4]);
  const T e5 = fma_t(P.dq[5], abs_t(r), P.dl[5]);
  // residual tau - C nu - D nu - g
  const T r0 = fma_t(-e0, u, fma_t(P.wmb, k0, fma_t(-q, aw, fma_t(r, av, tau[0]))));
  const T r1 = fma_t(-e1, v, fma_t(P.wmb, k1, fma_t(-r, au, fma_t(p, aw, tau[1]))));
  const T r2 = fma_t(-e2, w, fma_t(P.wmb, k2, fma_t(-p, av, fma_t(q, au, tau[2]))));
  const T r3 = fma_t(-e3, p, fma_t(-P.hz, k1,
                   fma_t(r, bq, fma_t(-q, br, fma_t(w, av, fma_t(-v, aw, tau[3]))))));
  const T r4 = fma_t(-e4, q, fma_t(P.hz, k0,
                   fma_t(p, br, fma_t(-r, bp, fma_t(u, aw, fma_t(-w, au, tau[4]))))));
  const T r5 = fma_t(-e5, r, fma_t(q, bp, fma_t(-p, bq, fma_t(v, au, fma_t(-u, av, tau[5])))));
  res[0] = r0; res[1] = r1; res[2] = r2; res[3] = r3; res[4] = r4; res[5] = r5;
}

template <class T>
__host__ __device__ __forceinline__ void rhs_residual(const T* x, T* xd, T (&res)[6],
                                                      const EnvConstT<T>& P, const T (&tau)[6]) {
  T mom[6];
  momentum(P, x + 7, mom);
  rhs_residual_m(x, mom, xd, res, P, tau);
}

template <class T>
__host__ __device__ __forceinline__ void rhs_core(const T* x, T* xd, const EnvConstT<T>& P,
                                                  const T (&tau)[6]) {
  T r[6];
  rhs_residual(x, xd, r, P, tau);
  // nu' = M^-1 r
  xd[7] = fma_t(P.Iuq, r[4], P.Iuu * r[0]);
  xd[8] = fma_t(P.Ivp, r[3], P.Ivv * r[1]);
  xd[9] = P.Iww * r[2];
  xd[10] = fma_t(P.Ipp, r[3], P.Ivp * r[1]);
  xd[11] = fma_t(P.Iqq, r[4], P.Iuq * r[0]);
  xd[12] = P.Irr * r[5];
}

// (h/2) M^-1 for the sub-step h: the structured inverse pre-scaled once per
// launch, so the RK4 stage velocities come from the residuals in FMAs alone
// (nu + (h/2) M^-1 r = nu + A r, nu + h M^-1 r = nu + 2 A r, and the
// combination (h/6) M^-1 (r1 + 2 r2 + 2 r3 + r4) = (1/3) A (...), M^-1 being
// constant over the sub-step).  The momenta follow without M: M (nu + c M^-1 r)
// = M nu + c r.
template <class T>
struct HalfInvT {
  T uu, vv, ww, pp, qq, rr, uq, vp;
};

template <class T>
__host__ __device__ __forceinline__ HalfInvT<T> half_step_inverse(const EnvConstT<T>& P, T h2) {
  HalfInvT<T> A;
  A.uu = h2 * P.Iuu; A.vv = h2 * P.Ivv; A.ww = h2 * P.Iww; A.pp = h2 * P.Ipp;
  A.qq = h2 * P.Iqq; A.rr = h2 * P.Irr; A.uq = h2 * P.Iuq; A.vp = h2 * P.Ivp;
  return A;
}

// y = base + A r
template <class T>
__host__ __device__ __forceinline__ void add_inv(const HalfInvT<T>& A, const T (&r)[6],
                                                 const T* base, T* y) {
  y[0] = fma_t(A.uu, r[0], fma_t(A.uq, r[4], base[0]));
  y[1] = fma_t(A.vv, r[1], fma_t(A.vp, r[3], base[1]));
  y[2] = fma_t(A.ww, r[2], base[2]);
  y[3] = fma_t(A.pp, r[3], fma_t(A.vp, r[1], base[3]));
  y[4] = fma_t(A.qq, r[4], fma_t(A.uq, r[0], base[4]));
  y[5] = fma_t(A.rr, r[5], base[5]);
}

// y = A r
template <class T>
__host__ __device__ __forceinline__ void mul_inv(const HalfInvT<T>& A, const T (&r)[6],
                                                 T (&y)[6]) {
  y[0] = fma_t(A.uu, r[0], A.uq * r[4]);
  y[1] = fma_t(A.vv, r[1], A.vp * r[3]);
  y[2] = A.ww * r[2];
  y[3] = fma_t(A.pp, r[3], A.vp * r[1]);
  y[4] = fma_t(A.qq, r[4], A.uq * r[0]);
  y[5] = A.rr * r[5];
}

// One classical RK4 sub-step (c = 0, 1/2, 1/2, 1; b = 1/6, 1/3, 1/3, 1/6) of
// the full state [p, q, nu, f], then q <- q / |q|.
//
// The thruster states enter only through the wrench B f and obey the linear
// lag f' = (f_cmd - f) / tau with f_cmd held, so their RK4 stage values are
// f_cmd + sigma_i (f - f_cmd) exactly (class constants), the stage wrenches
// are B f_cmd + sigma_i dg with dg = B (f - f_cmd), and the sub-step maps
// f - f_cmd and dg alike to rho times themselves: the same discrete map as
// generic RK4 on the lag states.  Over the S sub-steps of a control step
// f - f_cmd therefore shrinks by rho^S and dg by rho per sub-step, so
// begin_control_step forms dg once and sets the lag states to their
// end-of-control-step value f_cmd + rho^S (f - f_cmd) directly; the sub-step
// then touches neither the lag states nor the allocation matrix, only
// dg <- rho dg.  Without a lag the wrench is the command wrench B f_cmd
// throughout.
template <int N, class T>
__host__ __device__ __forceinline__ void lag_wrench(const ClassConst& cc, const T* x,
                                                    const T (&fcmd)[N], T (&dg)[6]) {
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    T s = mul_nc(T(cc.B[k][0]), x[13] - fcmd[0]);
#pragma unroll
    for (int i = 1; i < N; ++i) s = fma_t(T(cc.B[k][i]), x[13 + i] - fcmd[i], s);
    dg[k] = s;
  }
}

// Start of a control step with the commanded thrust f_cmd: dg = B (f - f_cmd)
// and f <- f_cmd + rho_s (f - f_cmd), rho_s = rho^S for the S sub-steps that
// follow (rho itself when one sub-step follows).
template <int N, bool LAG, class T>
__host__ __device__ __forceinline__ void begin_control_step(const ClassConst& cc, T* x,
                                                            const T (&fcmd)[N], T (&dg)[6],
                                                            T rho_s) {
  if constexpr (LAG) {
    lag_wrench<N>(cc, x, fcmd, dg);
#pragma unroll
    for (int i = 0; i < N; ++i) x[13 + i] = fma_t(rho_s, x[13 + i] - fcmd[i], fcmd[i]);
  } else {
#pragma unroll
    for (int k = 0; k < 6; ++k) dg[k] = T(0);
  }
}

// m is the momentum M nu of the state, carried from sub-step to sub-step of a
// control step (formed by control_step): the stage momenta are m + c r and
// the sub-step ends with m <- m + (h/6)(r1 + 2 r2 + 2 r3 + r4), equal to
// M nu of the new state in exact arithmetic.
template <int N, bool LAG, class T>
__host__ __device__ __forceinline__ void rk4_substep(T* x, T (&m)[6], const EnvConstT<T>& P,
                                                     const HalfInvT<T>& A, const T (&gcmd)[6],
                                                     T (&dg)[6], const StepConstT<T>& sc) {
  T tau[6];
  if constexpr (LAG) {
#pragma unroll
    for (int k = 0; k < 6; ++k) tau[k] = gcmd[k] + dg[k];
  } else {
#pragma unroll
    for (int k = 0; k < 6; ++k) tau[k] = gcmd[k];
  }
  // stage / combination factors of the kinematic rows; the quaternion rows of
  // rhs_residual are 2 q'.  The velocity rows go through A = (h/2) M^-1.
  auto f2 = [&](int i) { return (i >= 3) ? sc.h2q : sc.h2; };
  auto f1 = [&](int i) { return (i >= 3) ? sc.dtq : sc.dt; };
  auto f6 = [&](int i) { return (i >= 3) ? sc.h6q : sc.h6; };
  // acc: kinematic rates (rows 0..6) and residuals (rows 7..12) summed with
  // the RK4 weights 1, 2, 2, 1; ms: the stage momentum
  T k[7], r[6], X[13], acc[13], t[6], ms[6];
  rhs_residual_m(x, m, k, r, P, tau);
#pragma unroll
  for (int i = 0; i < 7; ++i) {
    acc[i] = k[i];
    X[i] = fma_t(f2(i), k[i], x[i]);
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    acc[7 + i] = r[i];
    ms[i] = fma_t(sc.h2, r[i], m[i]);
  }
  add_inv(A, r, x + 7, X + 7);
  if constexpr (LAG) {
#pragma unroll
    for (int j = 0; j < 6; ++j) tau[j] = fma_t(sc.s2, dg[j], gcmd[j]);
  }
  rhs_residual_m(X, ms, k, r, P, tau);
#pragma unroll
  for (int i = 0; i < 7; ++i) {
    acc[i] = fma_t(sc.two, k[i], acc[i]);
    X[i] = fma_t(f2(i), k[i], x[i]);
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    acc[7 + i] = fma_t(sc.two, r[i], acc[7 + i]);
    ms[i] = fma_t(sc.h2, r[i], m[i]);
  }
  add_inv(A, r, x + 7, X + 7);
  if constexpr (LAG) {
#pragma unroll
    for (int j = 0; j < 6; ++j) tau[j] = fma_t(sc.s3, dg[j], gcmd[j]);
  }
  rhs_residual_m(X, ms, k, r, P, tau);
#pragma unroll
  for (int i = 0; i < 7; ++i) {
    acc[i] = fma_t(sc.two, k[i], acc[i]);
    X[i] = fma_t(f1(i), k[i], x[i]);
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    acc[7 + i] = fma_t(sc.two, r[i], acc[7 + i]);
    ms[i] = fma_t(sc.dt, r[i], m[i]);
  }
  mul_inv(A, r, t);
#pragma unroll
  for (int i = 0; i < 6; ++i) X[7 + i] = fma_t(sc.two, t[i], x[7 + i]);
  if constexpr (LAG) {
#pragma unroll
    for (int j = 0; j < 6; ++j) tau[j] = fma_t(sc.s4, dg[j], gcmd[j]);
  }
  rhs_residual_m(X, ms, k, r, P, tau);
#pragma unroll
  for (int i = 0; i < 7; ++i) x[i] = fma_t(f6(i), acc[i] + k[i], x[i]);
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    r[i] += acc[7 + i];
    m[i] = fma_t(sc.h6, r[i], m[i]);
  }
  mul_inv(A, r, t);
#pragma unroll
  for (int i = 0; i < 6; ++i) x[7 + i] = fma_t(sc.third, t[i], x[7 + i]);
  if constexpr (LAG) {
#pragma unroll
    for (int k2 = 0; k2 < 6; ++k2) dg[k2] *= sc.rho;
  }
  const T n2 = x[3] * x[3] + x[4] * x[4] + x[5] * x[5] + x[6] * x[6];
  const T inv = rsqrt_t(n2);
  x[3] *= inv;
  x[4] *= inv;
  x[5] *= inv;
  x[6] *= inv;
}

// One control step: S sub-steps with the commanded thrust f_cmd (wrench gcmd)
// held; rho_s = rho^S.  MG_SUBSTEP_UNROLL sub-steps are unrolled per loop trip.
#ifndef MG_SUBSTEP_UNROLL
#define MG_SUBSTEP_UNROLL 1
#endif
#define MG_PRAGMA_(x) _Pragma(#x)
#define MG_UNROLL_(n) MG_PRAGMA_(unroll n)
template <int N, bool LAG, class T>
__host__ __device__ __forceinline__ void control_step(T* x, const EnvConstT<T>& P,
                                                      const HalfInvT<T>& A, const ClassConst& cc,
                                                      const T (&fcmd)[N], const T (&gcmd)[6],
                                                      const StepConstT<T>& sc, int S, T rho_s) {
  T dg[6], m[6];
  begin_control_step<N, LAG>(cc, x, fcmd, dg, rho_s);
  momentum(P, x + 7, m);
  MG_UNROLL_(MG_SUBSTEP_UNROLL)
  for (int s = 0; s < S; ++s) rk4_substep<N, LAG>(x, m, P, A, gcmd, dg, sc);
}

}  // namespace mg
