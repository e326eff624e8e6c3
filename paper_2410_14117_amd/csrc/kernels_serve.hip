// kernels_serve.hip -- device side of the continuous-batching serving loop:
// the join of admitted pages (state + per-env factorisation, tick-list entry),
// the tick that advances the active pages of every class by up to `steps`
// control steps (as many as each request has left), and the leave of finished
// pages (states into the tick's result staging, list entry emptied).
#include "fossen_device.h"

namespace mg {

// one block of 64 threads per admitted page
__global__ void __launch_bounds__(64) k_serve_join(const ServeInitItem* __restrict__ items,
                                                   ServeTickItem* __restrict__ list,
                                                   const ClassNominal* __restrict__ nominal,
                                                   int32_t Dmax, const DebugArgs dbg) {
  const ServeInitItem it = items[blockIdx.x];
  const int lane = threadIdx.x;
  if (lane == 0 && MG_CHECK_WITH(dbg, it.list_index >= 0 && it.list_index < dbg.list, kDbgList))
    list[it.list_index] = it.item;
  const int32_t col32 = it.cols_src[lane];
  it.cols[lane] = col32;
  const int64_t col = col32;
  if (col < 0) return;
  if (!MG_CHECK_WITH(dbg, col < it.ld, kDbgPage)) return;
  const ClassNominal& nom = nominal[it.cls];
  double prm[kNumParams];
#pragma unroll
  for (int i = 0; i < kNumParams; ++i) {
    double pi = nom.p[i];
    if (it.mult) pi *= (double)it.mult[i * it.ld + col];
    prm[i] = (double)(float)pi;
  }
  float dv[kNumDerived];
  derive_constants(prm, nom.zg, nom.zb, dv);
#pragma unroll
  for (int i = 0; i < kNumDerived; ++i) it.block[(Dmax + i) * kPageEnvs + lane] = dv[i];
  const int Dc = 13 + (nom.lag ? nom.n_thr : 0);
  for (int i = 0; i < Dmax; ++i)
    it.block[i * kPageEnvs + lane] = i < Dc ? it.x0[i * it.ld + col] : 0.0f;
}

// Output number k (0-based) of the SplitMix64 generator seeded with `seed`
// (Steele, Lea and Flood, "Fast splittable pseudorandom number generators",
// OOPSLA 2014): the mixing function applied to seed + (k + 1) * gamma.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// One page (64 envs, one per lane) of class constants cc: the request's
// control steps [first, first + cnt) with the state in registers throughout.
template <int N, bool LAG>
__device__ __forceinline__ void serve_page(const ServeTickItem& it, const ClassConst& cc,
                                           const ServeTickArgs& a, int lane) {
  constexpr int D = Dims<N, LAG>::D;
  const int64_t col = it.cols[lane];
  if (col < 0) return;
  if (!MG_CHECK(a, col < (it.actions ? it.ld : it.n), kDbgPage)) return;
  const StepConstT<float> sc = make_step_const(cc, a.dt);
  float x[D];
#pragma unroll
  for (int i = 0; i < D; ++i) x[i] = it.block[i * kPageEnvs + lane];
  const EnvConst P = load_env_const(it.block + a.Dmax * kPageEnvs, kPageEnvs, lane);
  const HalfInvT<float> A = half_step_inverse(P, sc.h2);
  // rows t < L only: a page whose request has done its L control steps and
  // waits in the list for room to retire gets cnt <= 0 and is left as it is
  const int64_t first = a.tick - it.t0;
  const int64_t left = (int64_t)it.L - first;
  const int64_t cnt = a.steps < left ? (int64_t)a.steps : left;
  for (int64_t k = 0; k < cnt; ++k) {
    float act[N], fcmd[N], gcmd[6];
    if (it.actions) {
      const float* af = it.actions + (first + k) * a.n_max * it.ld + col;
#pragma unroll
      for (int i = 0; i < N; ++i) act[i] = af[i * it.ld];
    } else {
      // throttle i of env col at control step t: generator output
      // (t * n_max + i) * n + col, its top 24 bits as u in [0, 1), 2 u - 1
      const uint64_t k0 = ((uint64_t)(first + k) * (uint64_t)a.n_max) * (uint64_t)it.n + col;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const uint64_t z = splitmix64_at(it.seed, k0 + (uint64_t)i * (uint64_t)it.n);
        act[i] = fmaf((float)(uint32_t)(z >> 40), 0x1p-23f, -1.0f);
      }
    }
    thrust_command<N>(cc, act, fcmd);
    command_wrench<N>(cc, fcmd, gcmd);
    // substeps is the server's S (cc.rho_s = rho^S) or, for the FIFO plain
    // baseline, 1 (rho)
    control_step<N, LAG>(x, P, A, cc, fcmd, gcmd, sc, a.substeps,
                         a.substeps == 1 ? cc.rho : cc.rho_s);
  }
#pragma unroll
  for (int i = 0; i < D; ++i) it.block[i * kPageEnvs + lane] = x[i];
}

// One wave per list entry over the entries of all classes (class c's entries
// follow those of classes 0..c-1); the wave's class picks the instantiation,
// so the classes' pages run side by side in one launch.
__global__ void __launch_bounds__(kBlock) k_serve_tick(const ServeTickArgs a) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int nwaves = (gridDim.x * blockDim.x) >> 6;
  int total = 0;
  for (int c = 0; c < a.n_classes; ++c) total += a.count[c];
  for (int e = wave; e < total; e += nwaves) {
    int c = 0, idx = e;
    while (idx >= a.count[c]) {
      idx -= a.count[c];
      ++c;
    }
    if (!MG_CHECK(a, idx < a.list_cap, kDbgList)) continue;
    const ServeTickItem it = a.list[(int64_t)c * a.list_cap + idx];
    if (!it.block) continue;
    const ClassConst& cc = a.cc[c];
    switch (cc.n_thr * 2 + (cc.lag ? 1 : 0)) {
#define MG_CASE(n)                                  \
  case 2 * n:                                       \
    serve_page<n, false>(it, cc, a, lane);          \
    break;                                          \
  case 2 * n + 1:                                   \
    serve_page<n, true>(it, cc, a, lane);           \
    break;
      MG_CASE(1) MG_CASE(2) MG_CASE(3) MG_CASE(4) MG_CASE(5) MG_CASE(6) MG_CASE(7) MG_CASE(8)
#undef MG_CASE
      default:
        break;
    }
  }
}

// one block of 64 threads per finished page
__global__ void __launch_bounds__(64) k_serve_leave(const ServeGatherItem* __restrict__ items,
                                                    ServeTickItem* __restrict__ list,
                                                    int32_t Dmax, const DebugArgs dbg) {
  const ServeGatherItem it = items[blockIdx.x];
  const int lane = threadIdx.x;
  if (lane == 0 && MG_CHECK_WITH(dbg, it.list_index >= 0 && it.list_index < dbg.list, kDbgList)) {
    ServeTickItem z;
    z.block = nullptr;
    z.cols = nullptr;
    z.actions = nullptr;
    z.ld = 0;
    z.t0 = 0;
    z.L = 0;
    z.pad_ = 0;
    z.seed = 0;
    z.n = 0;
    list[it.list_index] = z;
  }
  const int64_t col = it.cols[lane];
  if (col < 0) return;
  if (!MG_CHECK_WITH(dbg, col < it.n, kDbgPage)) return;
  for (int i = 0; i < Dmax; ++i) it.out[i * it.n + col] = it.block[i * kPageEnvs + lane];
}

hipError_t launch_serve_join(const ServeInitItem* items, int32_t n_items, ServeTickItem* list,
                             const ClassNominal* nominal, int32_t Dmax, const DebugArgs& dbg,
                             hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_serve_join, dim3(n_items), dim3(64), 0, s, items, list, nominal, Dmax,
                     dbg);
  return hipGetLastError();
}

hipError_t launch_serve_tick(const ServeTickArgs& a, int32_t grid, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_serve_tick, dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_serve_leave(const ServeGatherItem* items, int32_t n_items, ServeTickItem* list,
                              int32_t Dmax, const DebugArgs& dbg, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_serve_leave, dim3(n_items), dim3(64), 0, s, items, list, Dmax, dbg);
  return hipGetLastError();
}

}  // namespace mg
