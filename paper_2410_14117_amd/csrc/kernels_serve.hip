// kernels_serve.hip -- device side of the continuous-batching serving loop:
// page initialisation (state + per-env factorisation), the persistent tick
// that advances every active page by one control step, and the gather of a
// finished request's states into caller order.
#include "fossen_device.h"

namespace mg {

// one block of 64 threads per admitted page
__global__ void __launch_bounds__(64) k_serve_init(const ServeInitItem* __restrict__ items,
                                                   const ClassNominal* __restrict__ nominal,
                                                   int32_t Dmax) {
  const ServeInitItem it = items[blockIdx.x];
  const int lane = threadIdx.x;
  const int32_t col32 = it.cols_src[lane];
  it.cols[lane] = col32;
  const int64_t col = col32;
  if (col < 0) return;
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

template <int N, bool LAG>
__global__ void __launch_bounds__(kBlock) k_serve_tick(const ServeTickItem* __restrict__ items,
                                                       const ServeTickHeader* __restrict__ hdr,
                                                       int32_t cls, const ClassConst cc,
                                                       int32_t Dmax, int32_t n_max,
                                                       int32_t substeps, float dt) {
  constexpr int D = Dims<N, LAG>::D;
  const int lane = threadIdx.x & 63;
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int nwaves = (gridDim.x * blockDim.x) >> 6;
  const int n = hdr->count[cls];
  const int64_t tick = hdr->tick;
  const StepConstT<float> sc = make_step_const(cc, dt);
  for (int e = wave; e < n; e += nwaves) {
    const ServeTickItem it = items[e];
    if (!it.block) continue;
    const int64_t col = it.cols[lane];
    if (col < 0) continue;
    float x[D];
#pragma unroll
    for (int i = 0; i < D; ++i) x[i] = it.block[i * kPageEnvs + lane];
    const EnvConst P = load_env_const(it.block + Dmax * kPageEnvs, kPageEnvs, lane);
    const HalfInvT<float> A = half_step_inverse(P, sc.h2);
    const float* af = it.actions + (tick - it.t0) * n_max * it.ld + col;
    float act[N], fcmd[N], gcmd[6];
#pragma unroll
    for (int i = 0; i < N; ++i) act[i] = af[i * it.ld];
    thrust_command<N>(cc, act, fcmd);
    command_wrench<N>(cc, fcmd, gcmd);
    // substeps is the server's S (cc.rho_s = rho^S) or, for the FIFO plain
    // baseline, 1 (rho)
    control_step<N, LAG>(x, P, A, cc, fcmd, gcmd, sc, substeps, substeps == 1 ? cc.rho : cc.rho_s);
#pragma unroll
    for (int i = 0; i < D; ++i) it.block[i * kPageEnvs + lane] = x[i];
  }
}

__global__ void __launch_bounds__(256) k_serve_patch(const ServePatch* __restrict__ patches,
                                                     int32_t n, ServeTickItem* __restrict__ list) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) list[patches[i].index] = patches[i].item;
}

hipError_t launch_serve_patch(const ServePatch* patches, int32_t n, ServeTickItem* list,
                              hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_serve_patch, dim3((n + 255) / 256), dim3(256), 0, s, patches, n, list);
  return hipGetLastError();
}

__global__ void __launch_bounds__(64) k_serve_gather(const ServeGatherItem* __restrict__ items,
                                                     int32_t Dmax) {
  const ServeGatherItem it = items[blockIdx.x];
  const int lane = threadIdx.x;
  const int64_t col = it.cols[lane];
  if (col < 0) return;
  for (int i = 0; i < Dmax; ++i) it.out[i * it.n + col] = it.block[i * kPageEnvs + lane];
}

hipError_t launch_serve_init(const ServeInitItem* items, int32_t n_items,
                             const ClassNominal* nominal, int32_t Dmax, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_serve_init, dim3(n_items), dim3(64), 0, s, items, nominal, Dmax);
  return hipGetLastError();
}

template <int N, bool LAG>
static hipError_t tick_t(const ClassConst& cc, int32_t cls, const ServeTickItem* items,
                         const ServeTickHeader* hdr, int32_t Dmax, int32_t n_max,
                         int32_t substeps, float dt, int32_t grid, hipStream_t s) {
  hipLaunchKernelGGL((k_serve_tick<N, LAG>), dim3(grid), dim3(kBlock), 0, s, items, hdr, cls, cc,
                     Dmax, n_max, substeps, dt);
  return hipGetLastError();
}

hipError_t launch_serve_tick(const ClassConst& cc, int32_t cls, const ServeTickItem* items,
                             const ServeTickHeader* hdr, int32_t Dmax, int32_t n_max,
                             int32_t substeps, float dt, int32_t grid, hipStream_t s) {
  const bool lag = cc.lag != 0;
#define MG_CASE(n)                                                                            \
  case n:                                                                                     \
    return lag ? tick_t<n, true>(cc, cls, items, hdr, Dmax, n_max, substeps, dt, grid, s)     \
               : tick_t<n, false>(cc, cls, items, hdr, Dmax, n_max, substeps, dt, grid, s);
  switch (cc.n_thr) {
    MG_CASE(1) MG_CASE(2) MG_CASE(3) MG_CASE(4) MG_CASE(5) MG_CASE(6) MG_CASE(7) MG_CASE(8)
    default:
      return hipErrorInvalidValue;
  }
#undef MG_CASE
}

hipError_t launch_serve_gather(const ServeGatherItem* items, int32_t n_items, int32_t Dmax,
                               hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_serve_gather, dim3(n_items), dim3(64), 0, s, items, Dmax);
  return hipGetLastError();
}

}  // namespace mg
