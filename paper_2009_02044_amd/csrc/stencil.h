// Staple sums of the Wilson-action force (Sec. 3, eqs. lattice_1 and plaquette).
#pragma once
#include "lattice.h"

namespace gl {

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
    load_link(A, U, j, idx(g, xpimj), Vp);
    load_link(B, U, i, idx(g, xmj), Vp);
    load_link(C, U, j, idx(g, xmj), Vp);
    G::add_to(S, G::dag_mul(G::mul(B, A), C), w);
  }
  return S;
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
