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
//               Its per-env body is adj_bwd_env (fossen_adjoint.h).
#include "fossen_adjoint.h"

namespace mg {

// The forward is held to three resident waves per SIMD (168 VGPRs; the few
// values it then spills lie outside the control-step loop).  The backward
// kernel needs about 285-385 registers (VGPRs + AGPRs), one wave per SIMD; its
// WAVES = 2 instantiation has 256, which pays only when the launch has more
// waves than one per SIMD across the chip (launch_adj_t picks it then).  The
// two-wave recomputing sweeps keep the parameter adjoints in registers and
// spill 13-38 values inside the sub-step VJP; the two-wave trajectory-reading
// sweep keeps them in LDS (ThetaBarLds, 20 KiB per block) and spills nothing,
// where in registers it spilled 40-90 values.  (LDS accumulators in the
// recomputing sweeps removed their spills too, but cost more than the spills:
// 4.0 against 3.6 ms on 2^20 envs.)
#ifndef MG_ADJ_FWD_WAVES_PER_EU
#define MG_ADJ_FWD_WAVES_PER_EU 3
#endif
#if MG_ADJ_FWD_WAVES_PER_EU > 0
#define MG_ADJ_FWD_ATTR __attribute__((amdgpu_waves_per_eu(MG_ADJ_FWD_WAVES_PER_EU)))
#else
#define MG_ADJ_FWD_ATTR
#endif

template <int N, bool LAG>
__global__ void __launch_bounds__(kBlock) MG_ADJ_FWD_ATTR k_adj_fwd(const AdjArgs a, const ClassConst cc) {
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
    // checkpoints and trajectory rows are written once and read back only by
    // the backward, after the whole forward: non-temporal stores keep them
    // from displacing the throttle frames in the caches (2^20 envs: 2-4 %)
    if (t % a.ckpt_every == 0) {
      float* ck = a.ckpt + (int64_t)(t / a.ckpt_every) * a.D * a.E + c;
#pragma unroll
      for (int i = 0; i < D; ++i) __builtin_nontemporal_store(x[i], ck + i * a.E);
      for (int i = D; i < a.D; ++i) __builtin_nontemporal_store(0.0f, ck + i * a.E);
    }
    float fcmd[N], gcmd[6];
    thrust_command<N>(cc, act, fcmd);
    command_wrench<N>(cc, fcmd, gcmd);
    control_step<N, LAG>(x, P, A, cc, fcmd, gcmd, sc, a.substeps, cc.rho_s);
    if (a.traj) {
      float* tf = a.traj + (int64_t)t * a.D * a.E + c;
#pragma unroll
      for (int i = 0; i < D; ++i) __builtin_nontemporal_store(x[i], tf + i * a.E);
      for (int i = D; i < a.D; ++i) __builtin_nontemporal_store(0.0f, tf + i * a.E);
    }
  }
#pragma unroll
  for (int i = 0; i < D; ++i) a.state[i * a.Ep + j] = x[i];
}

template <int N, bool LAG, int WAVES, bool WHOLE, bool TRAJ = false>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(WAVES)))
k_adj_bwd(const AdjArgs a, const ClassConst cc) {
  const int64_t local = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (local >= a.seg_len) return;
  if (!MG_CHECK(a, a.seg_start + a.seg_len <= a.Ep, kDbgSegment)) return;
  const int64_t j = a.seg_start + local;
  const int64_t c = a.perm ? (int64_t)a.perm[j] : j;
  if (!MG_CHECK(a, c >= 0 && c < a.dbg.cols, kDbgColumn)) return;
  const EnvConst P = load_env_const(a.derived, a.Ep, j);
  const StepConstT<float> sc = make_step_const(cc, a.dt);
  const HalfInvT<float> A = half_step_inverse(P, sc.h2);
  if constexpr (WAVES == 1 || !TRAJ) {
    ThetaBar<float> thb;
    theta_bar_zero(thb);
    adj_bwd_env<N, LAG, WHOLE, WAVES == 1, TRAJ>(a, cc, P, sc, A, j, c, thb);
  } else {
    // two waves per SIMD, trajectory inputs: the parameter adjoints live in LDS
    __shared__ float thb_lds[20 * kBlock];
    adj_bwd_env<N, LAG, WHOLE, false, TRAJ>(a, cc, P, sc, A, j, c,
                                            theta_bar_lds(thb_lds + threadIdx.x));
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
  if (!MG_CHECK(a, a.seg_start + a.seg_len <= a.Ep, kDbgSegment)) return;
  const int64_t j = a.seg_start + local;
  const int64_t c = a.perm ? (int64_t)a.perm[j] : j;
  if (!MG_CHECK(a, c >= 0 && c < a.dbg.cols, kDbgColumn)) return;
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
  if (backward && a.recomputed == 2 && crowded)
    hipLaunchKernelGGL((k_adj_bwd<N, LAG, 2, true, true>), dim3((unsigned)nblk), dim3(kBlock), 0,
                       s, a, cc);
  else if (backward && a.recomputed == 2)
    hipLaunchKernelGGL((k_adj_bwd<N, LAG, 1, true, true>), dim3((unsigned)nblk), dim3(kBlock), 0,
                       s, a, cc);
  else if (backward && a.recomputed && crowded)
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
