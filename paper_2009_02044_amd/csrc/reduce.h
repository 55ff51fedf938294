// Per-site observable accumulators and their deterministic block reduction, shared by
// the observables kernel, the Gauss-residual kernel and the observing step kernel.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gl {

// slots: eps, p_L, p_T, S_L, |G|^2, |rho|^2, max|G^a|, max unitarity, nonfinite
constexpr int NQ = 9;
enum { Q_EPS = 0, Q_PL, Q_PT, Q_SL, Q_G2, Q_RHO2, Q_GMAX, Q_UNIT, Q_BAD };
__device__ __forceinline__ bool q_is_max(int q) { return q == Q_GMAX || q == Q_UNIT; }

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
  return v;
}

// Reduce the slots of acc selected by the bit mask over a work-group of BS threads
// (64-lane shuffles, then the wavefronts in a fixed order through LDS) and write them to
// dst[q]; the slots selected by the bit mask ADD are added to what dst already holds.  Every
// thread of the work-group must call it.
constexpr unsigned Q_ALL = (1u << NQ) - 1;
template <int BS, unsigned ADD = 0u>
__device__ __forceinline__ void block_reduce_write(const double (&acc)[NQ], unsigned mask, double* dst) {
  __shared__ double red[BS / 64][NQ];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    if (!((mask >> q) & 1u)) continue;
    const double v = q_is_max(q) ? wave_max(acc[q]) : wave_sum(acc[q]);
    if (lane == 0) red[wv][q] = v;
  }
  __syncthreads();
  if ((int)threadIdx.x < NQ && ((mask >> threadIdx.x) & 1u)) {
    const int q = threadIdx.x;
    double v = red[0][q];
    for (int w = 1; w < BS / 64; ++w) v = q_is_max(q) ? fmax(v, red[w][q]) : v + red[w][q];
    if ((ADD >> q) & 1u) v += dst[q];
    dst[q] = v;
  }
}

template <typename A> __device__ __forceinline__ double norm2(const A& a) {
  constexpr int NG = sizeof(a.c) / sizeof(a.c[0]);
  double s = 0;
#pragma unroll
  for (int k = 0; k < NG; ++k) s += (double)a.c[k] * (double)a.c[k];
  return s;
}

}  // namespace gl
