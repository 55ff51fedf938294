// Staple sums of the Wilson-action force (Sec. 3, eqs. lattice_1 and plaquette).
#pragma once
#include "lattice.h"

namespace gl {

// Optional scheduling fence between staples (limits how many links the compiler keeps
// in flight at once; a register-pressure / occupancy trade-off, off by default).
#ifndef GL_STAPLE_FENCE
#define GL_STAPLE_FENCE 1
#endif
__device__ __forceinline__ void staple_fence() {
#if GL_STAPLE_FENCE
  __builtin_amdgcn_sched_barrier(0);
#endif
}

// S = sum_{j != i} a_j^-2 [ U_j(x+i) U_i^dag(x+j) U_j^dag(x) + U_j^dag(x+i-j) U_i^dag(x-j) U_j(x-j) ]
// so that U_i(x) S = sum_{j != i} a_j^-2 (U_{i,j}(x) + U_{i,-j}(x)).  G is the group in
// the compute precision; the links are read from storage of type T.
template <typename G, typename T>
__device__ __forceinline__ typename G::Link staple_sum(const T* __restrict__ U, const Geom& g,
                                                       Site x, int i, const double* inv_a2) {
  using L = typename G::Link;
  using R = typename G::Real;
  L S = G::zero();
  const int64_t Vp = g.Vp;
  Site xpi = shifted(g, x, i, +1);
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    if (j == i) continue;
    const R w = (R)inv_a2[j];
    Site xpj = shifted(g, x, j, +1);
    Site xmj = shifted(g, x, j, -1);
    Site xpimj = shifted(g, xpi, j, -1);
    L A, B, C;
    load_link(A, U, j, idx(g, xpi), Vp);
    load_link(B, U, i, idx(g, xpj), Vp);
    load_link(C, U, j, idx(g, x), Vp);
    G::add_to(S, G::mul_dag(G::mul_dag(A, B), C), w);
    staple_fence();
    load_link(A, U, j, idx(g, xpimj), Vp);
    load_link(B, U, i, idx(g, xmj), Vp);
    load_link(C, U, j, idx(g, xmj), Vp);
    G::add_to(S, G::dag_mul(G::mul(B, A), C), w);
    staple_fence();
  }
  return S;
}

// The other two directions of i in increasing order.
GL_HD int other_lo(int i) { return i == 0 ? 1 : 0; }
GL_HD int other_hi(int i) { return i == 2 ? 1 : 2; }

// Staple sum of direction i for the step kernel.  With (j1, j2) = (other_lo(i),
// other_hi(i)) and w_j = a_j^-2 it returns
//   S = (w_j1 / w_j2) [fwd_j1 + bwd_j1] + [fwd_j2 + bwd_j2],
//   fwd_j = U_j(x+i) U_i^dag(x+j) U_j^dag(x),  bwd_j = U_j^dag(x+i-j) U_i^dag(x-j) U_j(x-j),
// so that sum_j w_j (U_{i,j} + U_{i,-j}) = w_j2 U_i(x) S.  The last product of every
// staple accumulates into S as one fused chain per entry, and a single scaling by
// ratio = w_j1 / w_j2 stands in for the per-staple weights.
// Link sources for the staple sums: fetch(l, d, s) sets l = U_d at site s.
template <typename T> struct GlobalLinks {
  const T* __restrict__ U;
  int64_t Vp;
  template <typename L> __device__ __forceinline__ void operator()(L& l, int d, uint32_t s) const {
    load_link(l, U, d, s, Vp);
  }
};

template <typename G, typename F>
__device__ __forceinline__ typename G::Link staple_sum_scaled_f(const F& fetch, const Geom& g, Site x, int i,
                                                                typename G::Real ratio) {
  using L = typename G::Link;
  L S;
  Site xpi = shifted(g, x, i, +1);
#pragma unroll
  for (int n = 0; n < 2; ++n) {
    const int j = n == 0 ? other_lo(i) : other_hi(i);
    Site xpj = shifted(g, x, j, +1);
    Site xmj = shifted(g, x, j, -1);
    Site xpimj = shifted(g, xpi, j, -1);
    L A, B, C;
    fetch(A, j, idx(g, xpi));
    fetch(B, i, idx(g, xpj));
    fetch(C, j, idx(g, x));
    const L P = G::mul_dag(A, B);
    if (n == 0) S = G::mul_dag(P, C);
    else G::acc_mul_dag(S, P, C);
    staple_fence();
    fetch(A, j, idx(g, xpimj));
    fetch(B, i, idx(g, xmj));
    fetch(C, j, idx(g, xmj));
    G::acc_dag_mul(S, G::mul(B, A), C);
    if (n == 0) G::scale(S, ratio);
    staple_fence();
  }
  return S;
}
template <typename G, typename T>
__device__ __forceinline__ typename G::Link staple_sum_scaled(const T* __restrict__ U, const Geom& g, Site x,
                                                              int i, typename G::Real ratio) {
  return staple_sum_scaled_f<G>(GlobalLinks<T>{U, g.Vp}, g, x, i, ratio);
}

// Forward plaquette U_{i,j}(x) = U_i(x) U_j(x+i) U_i^dag(x+j) U_j^dag(x) (eq. plaquette).
template <typename G, typename T>
__device__ __forceinline__ typename G::Link plaquette(const T* __restrict__ U, const Geom& g, Site x,
                                                      int i, int j) {
  using L = typename G::Link;
  const int64_t Vp = g.Vp;
  L Ui, A, B, C;
  load_link(Ui, U, i, idx(g, x), Vp);
  load_link(A, U, j, idx(g, shifted(g, x, i, +1)), Vp);
  load_link(B, U, i, idx(g, shifted(g, x, j, +1)), Vp);
  load_link(C, U, j, idx(g, x), Vp);
  return G::mul_dag(G::mul_dag(G::mul(Ui, A), B), C);
}

}  // namespace gl
