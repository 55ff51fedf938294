// Staple sums of the Wilson-action force (Sec. 3, eqs. lattice_1 and plaquette).
#pragma once
#include "lattice.h"

namespace gl {

// Optional scheduling fence between staples (limits how many links the compiler keeps
// in flight at once; a register-pressure / occupancy trade-off, off by default).
#ifndef GL_STAPLE_FENCE
#define GL_STAPLE_FENCE 0
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

// All three staple sums at once, visiting each unordered pair {i, j} once: the product
// P = U_j(x+i) U_i^dag(x+j) serves both forward staples, P U_j^dag(x) for direction i
// and P^dag U_i^dag(x) for direction j, and every neighbour link is loaded once per
// pair.  The own links arrive in Ux.
template <typename G, typename T>
__device__ __forceinline__ void staple_sums_pairs(const T* __restrict__ U, const Geom& g, Site x,
                                                  const typename G::Link (&Ux)[3], const double* inv_a2,
                                                  typename G::Link (&S)[3]) {
  using L = typename G::Link;
  using R = typename G::Real;
  const int64_t Vp = g.Vp;
#pragma unroll
  for (int i = 0; i < 3; ++i) S[i] = G::zero();
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i + 1; j < 3; ++j) {
      const R wi = (R)inv_a2[j], wj = (R)inv_a2[i];   // weight of the (i,j) plane in F_i and F_j
      Site xpi = shifted(g, x, i, +1), xpj = shifted(g, x, j, +1);
      {
        L A, B;
        load_link(A, U, j, idx(g, xpi), Vp);
        load_link(B, U, i, idx(g, xpj), Vp);
        L P = G::mul_dag(A, B);                        // U_j(x+i) U_i^dag(x+j)
        G::add_to(S[i], G::mul_dag(P, Ux[j]), wi);
        G::add_to(S[j], G::dag_mul(P, G::dag(Ux[i])), wj);
      }
      {
        // backward staple of direction i in the (i, -j) plane
        Site xmj = shifted(g, x, j, -1);
        L A, B, C;
        load_link(A, U, j, idx(g, shifted(g, xpi, j, -1)), Vp);
        load_link(B, U, i, idx(g, xmj), Vp);
        load_link(C, U, j, idx(g, xmj), Vp);
        G::add_to(S[i], G::dag_mul(G::mul(B, A), C), wi);
      }
      {
        // backward staple of direction j in the (j, -i) plane
        Site xmi = shifted(g, x, i, -1);
        L A, B, C;
        load_link(A, U, i, idx(g, shifted(g, xpj, i, -1)), Vp);
        load_link(B, U, j, idx(g, xmi), Vp);
        load_link(C, U, i, idx(g, xmi), Vp);
        G::add_to(S[j], G::dag_mul(G::mul(B, A), C), wj);
      }
    }
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
