// kernels_split.hip -- the split integration of Sec. II as a variant of the
// step: a physics engine advances the rigid body (M_RB, C_RB, g_RB) while the
// hydrodynamic wrench, computed from the current state, acts on it as an
// external force.  Per sub-step of dt:
//   tau_h = -M_A a_prev - C_A(nu) nu - D(nu) nu - g_A(eta)
//   a     = M_RB^-1 (tau_thrust + tau_h - C_RB(nu) nu - g_RB(eta))
//   nu <- nu + dt a;  p <- p + dt R(q) v;  q <- (q + dt/2 q (x) (0, w)) / |.|
//   f  <- f + dt (f_cmd - f) / tau_thr;  a_prev <- a
// Since C and g are linear in M and in (W, B), tau_h - C_RB nu - g_RB is the
// coupled residual tau - C(M) nu - D nu - g of the fused step minus
// M_A a_prev, so the residual code is shared.  One env per lane.
#include "fossen_device.h"

namespace mg {

namespace {

// M_RB^-1 for r_g on the z axis: (u, q) and (v, p) couple through m z_g.
struct RigidInv {
  float uu, vv, ww, pp, qq, rr, uq, vp;
};

__device__ __forceinline__ RigidInv rigid_inverse(const float* params, int64_t Ep, int64_t j,
                                                  double zg) {
  const double m = params[j], ix = params[Ep + j], iy = params[2 * Ep + j],
               iz = params[3 * Ep + j];
  const double mzz = mul_nc(mul_nc(m, zg), zg);
  const double mpp = ix + mzz, mqq = iy + mzz, muq = m * zg, mvp = -m * zg;
  const double det_uq = m * mqq - muq * muq, det_vp = m * mpp - mvp * mvp;
  RigidInv I;
  I.uu = (float)(mqq / det_uq);
  I.qq = (float)(m / det_uq);
  I.uq = (float)(-muq / det_uq);
  I.vv = (float)(mpp / det_vp);
  I.pp = (float)(m / det_vp);
  I.vp = (float)(-mvp / det_vp);
  I.ww = (float)(1.0 / m);
  I.rr = (float)(1.0 / iz);
  return I;
}

}  // namespace

template <int N, bool LAG>
__global__ void __launch_bounds__(kBlock) k_split(const SplitArgs a, const ClassConst cc) {
  constexpr int D = Dims<N, LAG>::D;
  const int64_t local = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (local >= a.seg_len) return;
  if (!MG_CHECK(a, a.seg_start + a.seg_len <= a.Ep, kDbgSegment)) return;
  const int64_t j = a.seg_start + local;
  const int64_t c = a.perm ? (int64_t)a.perm[j] : j;
  if (!MG_CHECK(a, c >= 0 && c < a.dbg.cols, kDbgColumn)) return;
  float x[D], acc[6], ma[6];
#pragma unroll
  for (int i = 0; i < D; ++i) x[i] = a.state[i * a.Ep + j];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    acc[i] = a.acc[i * a.Ep + j];
    ma[i] = a.params[(4 + i) * a.Ep + j];
  }
  const EnvConst P = load_env_const(a.derived, a.Ep, j);
  const RigidInv I = rigid_inverse(a.params, a.Ep, j, a.zg);
  const float dt = a.dt, hdt = 0.5f * a.dt, kdt = a.dt * cc.inv_tau;
  for (int t = 0; t < a.n_ctrl; ++t) {
    const float* af = a.actions + (int64_t)t * a.n_max * a.E + c;
    float act[N], fcmd[N], gcmd[6];
#pragma unroll
    for (int i = 0; i < N; ++i) act[i] = af[i * a.E];
    thrust_command<N>(cc, act, fcmd);
    command_wrench<N>(cc, fcmd, gcmd);
    for (int s = 0; s < a.substeps; ++s) {
      float tau[6];
      if constexpr (LAG) {
        float dg[6];
        lag_wrench<N>(cc, x, fcmd, dg);
#pragma unroll
        for (int k = 0; k < 6; ++k) tau[k] = gcmd[k] + dg[k];
      } else {
#pragma unroll
        for (int k = 0; k < 6; ++k) tau[k] = gcmd[k];
      }
      float kin[7], r[6];
      rhs_residual(x, kin, r, P, tau);
#pragma unroll
      for (int k = 0; k < 6; ++k) r[k] = fma_t(-ma[k], acc[k], r[k]);
      acc[0] = fma_t(I.uq, r[4], I.uu * r[0]);
      acc[1] = fma_t(I.vp, r[3], I.vv * r[1]);
      acc[2] = I.ww * r[2];
      acc[3] = fma_t(I.pp, r[3], I.vp * r[1]);
      acc[4] = fma_t(I.qq, r[4], I.uq * r[0]);
      acc[5] = I.rr * r[5];
#pragma unroll
      for (int k = 0; k < 6; ++k) x[7 + k] = fma_t(dt, acc[k], x[7 + k]);
      // p += dt R(q) v with R(q) v = v + q_w t + q_v x t, t = 2 q_v x v
      const float qw = x[3], qx = x[4], qy = x[5], qz = x[6];
      const float u = x[7], v = x[8], w = x[9], p = x[10], q = x[11], rr = x[12];
      const float t0 = 2.0f * (qy * w - qz * v), t1 = 2.0f * (qz * u - qx * w),
                  t2 = 2.0f * (qx * v - qy * u);
      x[0] = fma_t(dt, u + qw * t0 + (qy * t2 - qz * t1), x[0]);
      x[1] = fma_t(dt, v + qw * t1 + (qz * t0 - qx * t2), x[1]);
      x[2] = fma_t(dt, w + qw * t2 + (qx * t1 - qy * t0), x[2]);
      // q += dt/2 q (x) (0, omega), then renormalise
      const float nw = fma_t(-hdt, qx * p + qy * q + qz * rr, qw);
      const float nx = fma_t(hdt, qw * p + qy * rr - qz * q, qx);
      const float ny = fma_t(hdt, qw * q + qz * p - qx * rr, qy);
      const float nz = fma_t(hdt, qw * rr + qx * q - qy * p, qz);
      const float inv = rsqrt_t(nw * nw + nx * nx + ny * ny + nz * nz);
      x[3] = nw * inv;
      x[4] = nx * inv;
      x[5] = ny * inv;
      x[6] = nz * inv;
      if constexpr (LAG) {
#pragma unroll
        for (int i = 0; i < N; ++i) x[13 + i] = fma_t(kdt, fcmd[i] - x[13 + i], x[13 + i]);
      }
    }
    if (a.traj) {
      float* tf = a.traj + (int64_t)t * a.D * a.E + c;
#pragma unroll
      for (int i = 0; i < D; ++i) tf[i * a.E] = x[i];
      for (int i = D; i < a.D; ++i) tf[i * a.E] = 0.0f;
    }
  }
#pragma unroll
  for (int i = 0; i < D; ++i) a.state[i * a.Ep + j] = x[i];
#pragma unroll
  for (int i = 0; i < 6; ++i) a.acc[i * a.Ep + j] = acc[i];
}

template <int N, bool LAG>
static hipError_t launch_split_t(const ClassConst& cc, const SplitArgs& a, hipStream_t s) {
  const int64_t nblk = (a.seg_len + kBlock - 1) / kBlock;
  if (nblk == 0) return hipSuccess;
  hipLaunchKernelGGL((k_split<N, LAG>), dim3((unsigned)nblk), dim3(kBlock), 0, s, a, cc);
  return hipGetLastError();
}

hipError_t launch_split(const ClassConst& cc, const SplitArgs& a, hipStream_t s) {
  const bool lag = cc.lag != 0;
#define MG_CASE(n)                                                               \
  case n:                                                                        \
    return lag ? launch_split_t<n, true>(cc, a, s) : launch_split_t<n, false>(cc, a, s);
  switch (cc.n_thr) {
    MG_CASE(1) MG_CASE(2) MG_CASE(3) MG_CASE(4) MG_CASE(5) MG_CASE(6) MG_CASE(7) MG_CASE(8)
    default:
      return hipErrorInvalidValue;
  }
#undef MG_CASE
}

}  // namespace mg
