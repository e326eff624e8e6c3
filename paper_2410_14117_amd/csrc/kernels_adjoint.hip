// kernels_adjoint.hip -- discrete adjoint of a T-control-step rollout with
// segment checkpointing.
//
//   k_adj_fwd : T control steps in one launch (state in registers); stores the
//               state before every ckpt_every-th step and, optionally, the
//               trajectory.
//   k_adj_bwd : one lane per env walks the segments last to first: recomputes
//               the segment's sub-step states from its checkpoint into a
//               scratch buffer, then sweeps the sub-step VJPs backwards,
//               emitting dL/d throttle per step and accumulating dL/d theta.
#include "fossen_adjoint.h"

namespace mg {

// The forward is held to three resident waves per SIMD (168 VGPRs; the few
// values it then spills lie outside the control-step loop).  The backward
// kernel needs about 320 registers (VGPRs + AGPRs), one wave per SIMD; its
// WAVES = 2 instantiation is squeezed into 256 and spills about 50 values
// inside the sub-step VJP to scratch.  That pays only when the launch has more
// waves than one per SIMD across the chip (launch_adj_t picks it then).
#ifndef MG_ADJ_FWD_WAVES_PER_EU
#define MG_ADJ_FWD_WAVES_PER_EU 3
#endif
#if MG_ADJ_FWD_WAVES_PER_EU > 0
#define MG_ADJ_FWD_ATTR __attribute__((amdgpu_waves_per_eu(MG_ADJ_FWD_WAVES_PER_EU)))
#else
#define MG_ADJ_FWD_ATTR
#endif

template <int N>
__device__ __forceinline__ void load_command(const ClassConst& cc, const AdjArgs& a, int t,
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
// Used by k_adj_recompute only: k_adj_bwd keeps its own copy of this loop
// (see there).
template <int N, bool LAG>
__device__ __forceinline__ void recompute_segment(const AdjArgs& a, const ClassConst& cc,
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

template <int N, bool LAG>
__global__ void __launch_bounds__(kBlock) MG_ADJ_FWD_ATTR k_adj_fwd(const AdjArgs a, const ClassConst cc) {
  constexpr int D = Dims<N, LAG>::D;
  const int64_t local = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (local >= a.seg_len) return;
  const int64_t j = a.seg_start + local;
  const int64_t c = a.perm ? (int64_t)a.perm[j] : j;
  float x[D];
#pragma unroll
  for (int i = 0; i < D; ++i) x[i] = a.state[i * a.Ep + j];
  const EnvConst P = load_env_const(a.derived, a.Ep, j);
  const StepConstT<float> sc = make_step_const(cc, a.dt);
  const HalfInvT<float> A = half_step_inverse(P, sc.h2);
  // each control step's throttles are loaded one step ahead, so that their
  // latency hides behind the current step's sub-steps (a launch with few waves
  // per SIMD has nothing else to hide it behind)
  const float* abase = a.actions + c;
  const int64_t frame = (int64_t)a.n_max * a.E;
  float nxt[N];
#pragma unroll
  for (int i = 0; i < N; ++i) nxt[i] = abase[i * a.E];
  for (int t = 0; t < a.T; ++t) {
    float act[N];
#pragma unroll
    for (int i = 0; i < N; ++i) act[i] = nxt[i];
    if (t + 1 < a.T) {
      const float* af = abase + (int64_t)(t + 1) * frame;
#pragma unroll
      for (int i = 0; i < N; ++i) nxt[i] = af[i * a.E];
    }
    if (t % a.ckpt_every == 0) {
      float* ck = a.ckpt + (int64_t)(t / a.ckpt_every) * a.D * a.E + c;
#pragma unroll
      for (int i = 0; i < D; ++i) ck[i * a.E] = x[i];
      for (int i = D; i < a.D; ++i) ck[i * a.E] = 0.0f;
    }
    float fcmd[N], gcmd[6];
    thrust_command<N>(cc, act, fcmd);
    command_wrench<N>(cc, fcmd, gcmd);
    control_step<N, LAG>(x, P, A, cc, fcmd, gcmd, sc, a.substeps, cc.rho_s);
    if (a.traj) {
      float* tf = a.traj + (int64_t)t * a.D * a.E + c;
#pragma unroll
      for (int i = 0; i < D; ++i) tf[i * a.E] = x[i];
      for (int i = D; i < a.D; ++i) tf[i * a.E] = 0.0f;
    }
  }
#pragma unroll
  for (int i = 0; i < D; ++i) a.state[i * a.Ep + j] = x[i];
}

// WHOLE: the sub-step inputs of the whole rollout are already in segbuf
// (k_adj_recompute); otherwise each segment is recomputed here, into a
// segment-sized segbuf, just before its sweep.  The recomputation loop is
// written out here rather than calling recompute_segment: with that call
// inlined, the one-wave 8-thruster lag instantiation (256 VGPRs + AGPRs)
// returned gradients 5e-2 away from the oracle's although the source was
// equivalent, and out of line the call's register saves made the kernel 2-3x
// slower; this loop, unchanged, matches the oracle to 5e-7.
template <int N, bool LAG, int WAVES, bool WHOLE>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(WAVES)))
k_adj_bwd(const AdjArgs a, const ClassConst cc) {
  constexpr int D = Dims<N, LAG>::D;
  const int64_t local = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (local >= a.seg_len) return;
  const int64_t j = a.seg_start + local;
  const int64_t c = a.perm ? (int64_t)a.perm[j] : j;
  const EnvConst P = load_env_const(a.derived, a.Ep, j);
  const StepConstT<float> sc = make_step_const(cc, a.dt);
  const HalfInvT<float> A = half_step_inverse(P, sc.h2);
  const int K = a.ckpt_every, S = a.substeps;
  const int nseg = (a.T + K - 1) / K;
  float lam[D];
#pragma unroll
  for (int i = 0; i < D; ++i) lam[i] = 0.0f;
  ThetaBar<float> thb;
  theta_bar_zero(thb);
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
      for (int s = S - 1; s >= 0; --s) {
        float y[D];
        const float* sb = a.segbuf + (int64_t)((t - base) * S + s) * D * a.Ep + j;
#pragma unroll
        for (int i = 0; i < D; ++i) y[i] = sb[i * a.Ep];
        rk4_substep_vjp<N, LAG>(y, P, cc, fcmd, gcmd, a.dt, lam, fcb, gcb, thb);
      }
      throttle_vjp<N>(cc, act, fcb, gcb, ab);
      float* ga = a.gact + (int64_t)t * a.n_max * a.E + c;
#pragma unroll
      for (int i = 0; i < N; ++i) ga[i * a.E] = ab[i];
      for (int i = N; i < a.n_max; ++i) ga[i * a.E] = 0.0f;
    }
  }
  // theta = (M_A(6), D_L(6), D_Q(6), B);  W - B and h_z = W z_g - B z_b carry B
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    a.gtheta[i * a.E + c] = thb.ma[i];
    a.gtheta[(6 + i) * a.E + c] = thb.dl[i];
    a.gtheta[(12 + i) * a.E + c] = thb.dq[i];
  }
  a.gtheta[18 * a.E + c] = -thb.wmb - a.zb * thb.hz;
  if (a.gx0) {
#pragma unroll
    for (int i = 0; i < D; ++i) a.gx0[i * a.E + c] = lam[i];
    for (int i = D; i < a.D; ++i) a.gx0[i * a.E + c] = 0.0f;
  }
}

// Every segment's recomputation at once (blockIdx.y = segment) into the
// whole-rollout buffer, ahead of a backward launch with a.recomputed: the
// segments' recomputations, independent of one another, then cost one
// segment's latency when the backward launch has few waves, and the sweep
// kernel carries no recomputation registers when it has many.
template <int N, bool LAG>
__global__ void __launch_bounds__(kBlock) MG_ADJ_FWD_ATTR k_adj_recompute(const AdjArgs a,
                                                                         const ClassConst cc) {
  constexpr int D = Dims<N, LAG>::D;
  const int64_t local = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (local >= a.seg_len) return;
  const int64_t j = a.seg_start + local;
  const int64_t c = a.perm ? (int64_t)a.perm[j] : j;
  const int seg = blockIdx.y;
  const int t0 = seg * a.ckpt_every, t1 = min(a.T, t0 + a.ckpt_every);
  const EnvConst P = load_env_const(a.derived, a.Ep, j);
  const StepConstT<float> sc = make_step_const(cc, a.dt);
  const HalfInvT<float> A = half_step_inverse(P, sc.h2);
  float x[D];
  const float* ck = a.ckpt + (int64_t)seg * a.D * a.E + c;
#pragma unroll
  for (int i = 0; i < D; ++i) x[i] = ck[i * a.E];
  recompute_segment<N, LAG>(a, cc, P, A, sc, x, t0, t1, 0, j, c);
}

template <int N, bool LAG>
static hipError_t launch_adj_recompute_t(const ClassConst& cc, const AdjArgs& a, hipStream_t s) {
  const int64_t nblk = (a.seg_len + kBlock - 1) / kBlock;
  const int nseg = (a.T + a.ckpt_every - 1) / a.ckpt_every;
  if (nblk == 0) return hipSuccess;
  hipLaunchKernelGGL((k_adj_recompute<N, LAG>), dim3((unsigned)nblk, (unsigned)nseg), dim3(kBlock),
                     0, s, a, cc);
  return hipGetLastError();
}

hipError_t launch_adj_recompute(const ClassConst& cc, const AdjArgs& a, hipStream_t s) {
  const bool lag = cc.lag != 0;
#define MG_CASE(n)                                                                     \
  case n:                                                                              \
    return lag ? launch_adj_recompute_t<n, true>(cc, a, s)                             \
               : launch_adj_recompute_t<n, false>(cc, a, s);
  switch (cc.n_thr) {
    MG_CASE(1) MG_CASE(2) MG_CASE(3) MG_CASE(4) MG_CASE(5) MG_CASE(6) MG_CASE(7) MG_CASE(8)
    default:
      return hipErrorInvalidValue;
  }
#undef MG_CASE
}

template <int N, bool LAG>
static hipError_t launch_adj_t(bool backward, const ClassConst& cc, const AdjArgs& a,
                               hipStream_t s) {
  const int64_t nblk = (a.seg_len + kBlock - 1) / kBlock;
  if (nblk == 0) return hipSuccess;
  // one wave per SIMD over the whole device: n_cu CUs x 4 SIMDs x 64 lanes
  const bool crowded = a.seg_len > (int64_t)a.n_cu * 4 * 64;
  if (backward && a.recomputed && crowded)
    hipLaunchKernelGGL((k_adj_bwd<N, LAG, 2, true>), dim3((unsigned)nblk), dim3(kBlock), 0, s, a,
                       cc);
  else if (backward && a.recomputed)
    hipLaunchKernelGGL((k_adj_bwd<N, LAG, 1, true>), dim3((unsigned)nblk), dim3(kBlock), 0, s, a,
                       cc);
  else if (backward && crowded)
    hipLaunchKernelGGL((k_adj_bwd<N, LAG, 2, false>), dim3((unsigned)nblk), dim3(kBlock), 0, s, a,
                       cc);
  else if (backward)
    hipLaunchKernelGGL((k_adj_bwd<N, LAG, 1, false>), dim3((unsigned)nblk), dim3(kBlock), 0, s, a,
                       cc);
  else
    hipLaunchKernelGGL((k_adj_fwd<N, LAG>), dim3((unsigned)nblk), dim3(kBlock), 0, s, a, cc);
  return hipGetLastError();
}

hipError_t launch_adjoint(bool backward, const ClassConst& cc, const AdjArgs& a, hipStream_t s) {
  const bool lag = cc.lag != 0;
#define MG_CASE(n)                                                                    \
  case n:                                                                             \
    return lag ? launch_adj_t<n, true>(backward, cc, a, s)                            \
               : launch_adj_t<n, false>(backward, cc, a, s);
  switch (cc.n_thr) {
    MG_CASE(1) MG_CASE(2) MG_CASE(3) MG_CASE(4) MG_CASE(5) MG_CASE(6) MG_CASE(7) MG_CASE(8)
    default:
      return hipErrorInvalidValue;
  }
#undef MG_CASE
}

}  // namespace mg
