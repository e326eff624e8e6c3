// kernels_step.hip -- reset (per-env factorisation), fused / plain step,
// deterministic episode statistics, and layout gather/scatter kernels.
#include "fossen_device.h"

namespace mg {

// ---------------------------------------------------------------------------
// statistics: wavefront butterfly -> one partial per block (fixed order)
// ---------------------------------------------------------------------------

__device__ __forceinline__ void block_stats(double s_dist, double m_dist, double s_ke,
                                            double n_bad, double* __restrict__ out) {
  __shared__ double sh[kBlock / 64][4];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    s_dist += __shfl_xor(s_dist, off, 64);
    m_dist = fmax(m_dist, __shfl_xor(m_dist, off, 64));
    s_ke += __shfl_xor(s_ke, off, 64);
    n_bad += __shfl_xor(n_bad, off, 64);
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
    sh[wave][0] = s_dist;
    sh[wave][1] = m_dist;
    sh[wave][2] = s_ke;
    sh[wave][3] = n_bad;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    const int k = threadIdx.x;
    double acc = sh[0][k];
#pragma unroll
    for (int wv = 1; wv < kBlock / 64; ++wv) acc = (k == 1) ? fmax(acc, sh[wv][k]) : acc + sh[wv][k];
    out[k] = acc;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// the step kernel: n_ctrl control steps x substeps RK4 sub-steps per launch,
// state and per-env constants in registers throughout; one env per lane.
// PLAIN instantiations do exactly one sub-step of one control step per launch
// (the per-sub-step comparator whose state round-trips HBM).
// ---------------------------------------------------------------------------

#ifndef MG_STEP_WAVES_PER_EU
#define MG_STEP_WAVES_PER_EU 0
#endif
#if MG_STEP_WAVES_PER_EU > 0
#define MG_STEP_ATTR __attribute__((amdgpu_waves_per_eu(MG_STEP_WAVES_PER_EU)))
#else
#define MG_STEP_ATTR
#endif

template <int N, bool LAG, bool PLAIN>
__global__ void __launch_bounds__(kBlock) MG_STEP_ATTR k_step(const StepArgs a, const ClassConst cc) {
  constexpr int D = Dims<N, LAG>::D;
  const int n_ctrl = PLAIN ? 1 : a.n_ctrl;
  const int substeps = PLAIN ? 1 : a.substeps;
  const int64_t local = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  bool active = local < a.seg_len &&
                MG_CHECK(a, a.seg_start + a.seg_len <= a.Ep, kDbgSegment);
  const int64_t j = a.seg_start + (active ? local : 0);
  // byte offsets of the lane's env in internal and caller rows (rows of at most
  // 2^30 floats, checked by the launcher): every access below is a wave-uniform
  // row pointer plus this 32-bit offset, which the compiler addresses as an
  // SGPR base plus a VGPR offset, with no per-access 64-bit index arithmetic
  const uint32_t jo = (uint32_t)j * 4u;
  int64_t c = active ? (a.perm ? (int64_t)lane_elem(a.perm, jo) : j) : 0;
  active = active && MG_CHECK(a, c >= 0 && c < a.dbg.cols, kDbgColumn);
  c = active ? c : 0;
  const uint32_t co = (uint32_t)c * 4u;

  float x[D];
  EnvConst P;
  // an env whose flags are set is frozen: it is not stepped; an env whose
  // state is non-finite at the end of the launch gets its launch-input state
  // back and is flagged, so that it is frozen from the next launch on
  bool frozen = false;
  if (active) {
#pragma unroll
    for (int i = 0; i < D; ++i) x[i] = lane_elem(a.state + i * a.Ep, jo);
    P = load_env_const_off(a.derived, a.Ep, jo);
    frozen = lane_elem(a.flags, (uint32_t)j) != 0;
  }
  const StepConstT<float> sc = make_step_const(cc, a.dt);
  const HalfInvT<float> A = half_step_inverse(P, sc.h2);
  for (int t = 0; t < n_ctrl; ++t) {
    double s_dist = 0.0, m_dist = 0.0, s_ke = 0.0, n_bad = 0.0;
    if (active) {
      const float* af = a.actions + (int64_t)t * a.n_max * a.E;
      float act[N], fcmd[N], gcmd[6];
#pragma unroll
      for (int i = 0; i < N; ++i) act[i] = lane_elem(af + i * a.E, co);
      thrust_command<N>(cc, act, fcmd);
      command_wrench<N>(cc, fcmd, gcmd);
      if (!frozen)
        control_step<N, LAG>(x, P, A, cc, fcmd, gcmd, sc, substeps, PLAIN ? cc.rho : cc.rho_s);
      if (a.traj) {
        float* tf = a.traj + (int64_t)t * a.D * a.E;
#pragma unroll
        for (int i = 0; i < D; ++i) lane_elem(tf + i * a.E, co) = x[i];
        for (int i = D; i < a.D; ++i) lane_elem(tf + i * a.E, co) = 0.0f;
      }
      if (a.partials) {
        bool finite = !frozen;
#pragma unroll
        for (int i = 0; i < D; ++i) finite = finite && isfinite(x[i]);
        if (finite) {
          float tx = 0.f, ty = 0.f, tz = 0.f;
          if (a.targets) {
            tx = lane_elem(a.targets, co);
            ty = lane_elem(a.targets + a.E, co);
            tz = lane_elem(a.targets + 2 * a.E, co);
          }
          const double dx = (double)x[0] - tx, dy = (double)x[1] - ty, dz = (double)x[2] - tz;
          s_dist = sqrt(dx * dx + dy * dy + dz * dz);
          m_dist = s_dist;
          // 1/2 nu^T M nu = 1/2 (v . a + w . b)
          const double u = x[7], v = x[8], w = x[9], p = x[10], q = x[11], r = x[12];
          const double au = (double)P.Muu * u + (double)P.Muq * q;
          const double av = (double)P.Mvv * v + (double)P.Mvp * p;
          const double aw = (double)P.Mww * w;
          const double bp = (double)P.Mvp * v + (double)P.Mpp * p;
          const double bq = (double)P.Muq * u + (double)P.Mqq * q;
          const double br = (double)P.Mrr * r;
          s_ke = 0.5 * (u * au + v * av + w * aw + p * bp + q * bq + r * br);
        } else {
          n_bad = 1.0;
        }
      }
    }
    if (a.partials)
      block_stats(s_dist, m_dist, s_ke, n_bad,
                  a.partials + ((int64_t)t * a.nblk_total + a.blk_off + blockIdx.x) * 4);
  }
  if (active) {
    bool finite = true;
#pragma unroll
    for (int i = 0; i < D; ++i) finite = finite && isfinite(x[i]);
    if (finite) {
#pragma unroll
      for (int i = 0; i < D; ++i) lane_elem(a.state + i * a.Ep, jo) = x[i];
    } else {
      // the launch-input state stays in place
      lane_elem(a.flags, (uint32_t)j) =
          (uint8_t)(lane_elem(a.flags, (uint32_t)j) | kFlagNonFinite);
    }
  }
}

template <int N, bool LAG>
static hipError_t launch_step_t(const ClassConst& cc, const StepArgs& a, hipStream_t s) {
  const int64_t nblk = (a.seg_len + kBlock - 1) / kBlock;
  if (nblk == 0) return hipSuccess;
  // 32-bit lane offsets (mg_create caps n_envs below 2^30)
  if (a.Ep > ((int64_t)1 << 30) || a.E > ((int64_t)1 << 30)) return hipErrorInvalidValue;
  if (a.n_ctrl == 1 && a.substeps == 1)
    hipLaunchKernelGGL((k_step<N, LAG, true>), dim3((unsigned)nblk), dim3(kBlock), 0, s, a, cc);
  else
    hipLaunchKernelGGL((k_step<N, LAG, false>), dim3((unsigned)nblk), dim3(kBlock), 0, s, a, cc);
  return hipGetLastError();
}

hipError_t launch_step(const ClassConst& cc, const StepArgs& a, hipStream_t s) {
  const bool lag = cc.lag != 0;
#define MG_CASE(n)                                                         \
  case n:                                                                  \
    return lag ? launch_step_t<n, true>(cc, a, s) : launch_step_t<n, false>(cc, a, s);
  switch (cc.n_thr) {
    MG_CASE(1) MG_CASE(2) MG_CASE(3) MG_CASE(4) MG_CASE(5) MG_CASE(6) MG_CASE(7) MG_CASE(8)
    default:
      return hipErrorInvalidValue;
  }
#undef MG_CASE
}

// second pass: stats[t] = fixed-order combination of the per-block partials
__global__ void __launch_bounds__(256) k_stats_finalize(const double* __restrict__ partials,
                                                        int32_t nblk, double* __restrict__ stats) {
  const int t = blockIdx.x;
  const double* p = partials + (int64_t)t * nblk * 4;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblk; b += 256) {
    v[0] += p[b * 4 + 0];
    v[1] = fmax(v[1], p[b * 4 + 1]);
    v[2] += p[b * 4 + 2];
    v[3] += p[b * 4 + 3];
  }
  __shared__ double sh[256][4];
#pragma unroll
  for (int k = 0; k < 4; ++k) sh[threadIdx.x][k] = v[k];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sh[threadIdx.x][0] += sh[threadIdx.x + w][0];
      sh[threadIdx.x][1] = fmax(sh[threadIdx.x][1], sh[threadIdx.x + w][1]);
      sh[threadIdx.x][2] += sh[threadIdx.x + w][2];
      sh[threadIdx.x][3] += sh[threadIdx.x + w][3];
    }
    __syncthreads();
  }
  if (threadIdx.x < 4) stats[t * 4 + threadIdx.x] = sh[0][threadIdx.x];
}

hipError_t launch_stats_finalize(const double* partials, int32_t nblk, int32_t n_ctrl,
                                 double* stats, hipStream_t s) {
  if (n_ctrl <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_stats_finalize, dim3(n_ctrl), dim3(256), 0, s, partials, nblk, stats);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// reset: parameters (nominal x multiplier, or absolute), the per-env
// factorisation of M = M_RB + M_A (FP64, rounded once), and the state
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) k_reset(const ResetArgs a) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.n) return;
  const int64_t id = a.ids ? a.ids[k] : k;
  if (id < 0 || id >= a.E) return;   // out-of-range ids are skipped (documented)
  if (!MG_CHECK(a, id < a.dbg.cols, kDbgColumn)) return;
  const int64_t j = a.iperm ? (int64_t)a.iperm[id] : id;
  if (!MG_CHECK(a, j >= 0 && j < a.Ep, kDbgInternal)) return;
  const ClassNominal& nom = a.nominal[a.class_of[j]];
  const bool spd = set_env_params(nom, a.param_in ? a.param_in + k : nullptr, a.n,
                                  a.param_absolute != 0, a.params, a.derived, a.Ep, j);
  if (a.flags) {
    const uint8_t keep = a.write_state ? 0 : (uint8_t)(a.flags[j] & kFlagNonFinite);
    a.flags[j] = (uint8_t)(keep | (spd ? 0 : kFlagNotSPD));
  }
  if (a.write_state && a.task_k) a.task_k[j] = 0;
  if (a.write_state && a.split_acc)
    for (int i = 0; i < 6; ++i) a.split_acc[i * a.Ep + j] = 0.0f;

  if (a.write_state) {
    const int Dc = 13 + (nom.lag ? nom.n_thr : 0);
    for (int i = 0; i < a.D; ++i) {
      float xi;
      if (i >= Dc) xi = 0.0f;
      else if (a.state_in) xi = a.state_in[i * a.n + k];
      else xi = (i == 3) ? 1.0f : 0.0f;
      a.state[i * a.Ep + j] = xi;
    }
  }
}

hipError_t launch_reset(const ResetArgs& a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  const int64_t nblk = (a.n + 255) / 256;
  hipLaunchKernelGGL(k_reset, dim3((unsigned)nblk), dim3(256), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// internal <-> caller order
// ---------------------------------------------------------------------------

__global__ void k_gather_out(const float* __restrict__ in, int64_t Ep, float* __restrict__ out,
                             int64_t E, int32_t rows, const int32_t* __restrict__ perm,
                             int64_t n_internal) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_internal) return;
  const int64_t c = perm ? (int64_t)perm[j] : j;
  if (c < 0 || c >= E) return;
  for (int r = 0; r < rows; ++r) out[r * E + c] = in[r * Ep + j];
}

__global__ void k_scatter_in(const float* __restrict__ in, int64_t E, float* __restrict__ out,
                             int64_t Ep, int32_t rows, const int32_t* __restrict__ perm,
                             int64_t n_internal) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_internal) return;
  const int64_t c = perm ? (int64_t)perm[j] : j;
  if (c < 0 || c >= E) return;
  for (int r = 0; r < rows; ++r) out[r * Ep + j] = in[r * E + c];
}

// status flags, internal bytes -> caller int32
__global__ void k_flags_out(const uint8_t* __restrict__ flags, int32_t* __restrict__ out,
                            int64_t E, const int32_t* __restrict__ perm, int64_t n_internal) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_internal) return;
  const int64_t c = perm ? (int64_t)perm[j] : j;
  if (c < 0 || c >= E) return;
  out[c] = flags[j];
}

// flags &= mask for every env
__global__ void k_flags_mask(uint8_t* __restrict__ flags, int64_t n, uint8_t mask) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) flags[j] = (uint8_t)(flags[j] & mask);
}

hipError_t launch_flags_out(const uint8_t* flags, int32_t* out, int64_t E, const int32_t* perm,
                            int64_t n_internal, hipStream_t s) {
  if (n_internal <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_flags_out, dim3((unsigned)((n_internal + 255) / 256)), dim3(256), 0, s,
                     flags, out, E, perm, n_internal);
  return hipGetLastError();
}

hipError_t launch_flags_mask(uint8_t* flags, int64_t n, uint8_t mask, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_flags_mask, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, flags, n,
                     mask);
  return hipGetLastError();
}

hipError_t launch_gather_out(const float* in, int64_t Ep, float* out, int64_t E, int32_t rows,
                             const int32_t* perm, int64_t n_internal, hipStream_t s) {
  if (n_internal <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_out, dim3((unsigned)((n_internal + 255) / 256)), dim3(256), 0, s,
                     in, Ep, out, E, rows, perm, n_internal);
  return hipGetLastError();
}

hipError_t launch_scatter_in(const float* in, int64_t E, float* out, int64_t Ep, int32_t rows,
                             const int32_t* perm, int64_t n_internal, hipStream_t s) {
  if (n_internal <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_in, dim3((unsigned)((n_internal + 255) / 256)), dim3(256), 0, s,
                     in, E, out, Ep, rows, perm, n_internal);
  return hipGetLastError();
}

}  // namespace mg
