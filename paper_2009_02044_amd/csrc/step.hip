// Leapfrog step with the CPIC charge hop (Sec. 3: eqs. lattice_1, lattice_2,
// plaquette, continuity and the nearest-grid-point transport rule).
//
// One thread owns one site x and its three links.  For each direction i it forms
// the staple sum
//   S_i = sum_{j != i} a_j^-2 [ U_j(x+i) U_i^dag(x+j) U_j^dag(x)
//                               + U_j^dag(x+i-j) U_i^dag(x-j) U_j(x-j) ],
// so that U_i(x) S_i = sum_j a_j^-2 (U_{i,j} + U_{i,-j}), and updates
//   E_i += dt ( -(1/a_i) proj(U_i S_i) + j_i ),   U_i' = exp(i a_i dt E_i) U_i,
// writing U' into the second link buffer (old links stay readable by the
// neighbours) and E in place.  On a hop step the z-link thread also moves both
// charge populations one cell with parallel transport and adds the current that
// satisfies the continuity equation exactly:
//   B (+z): rho_B(x+z) <- U_z^dag(x) rho_B(x) U_z(x),     j_z(x) -= (a_L/dt) rho_B(x)
//   A (-z): rho_A(x)   <- U_z(x) rho_A(x+z) U_z^dag(x),   j_z(x) += (a_L/dt) rho_A'(x)
// With co-moving charge storage both rewrites are in place (one slot per thread).
#include "internal.h"
#include "stencil.h"

namespace gl {

template <typename G, typename T, bool HOP>
__global__ void __launch_bounds__(256) k_leapfrog(const T* __restrict__ U, T* __restrict__ Unew,
                                                  T* __restrict__ E, T* __restrict__ rhoA,
                                                  T* __restrict__ rhoB, Geom g, StepConst c) {
  using L = typename G::Link;
  using A = typename G::Alg;
  constexpr int NG = G::NG;
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  const int64_t V = g.V;
  Site x;
  x.x = (int)(s % g.nt);
  x.y = (int)((s / g.nt) % g.nt);
  x.z = (int)(s / g.layer);
  const double inv_a2[3] = {1.0 / (c.a[0] * c.a[0]), 1.0 / (c.a[1] * c.a[1]), 1.0 / (c.a[2] * c.a[2])};
#pragma unroll 1
  for (int i = 0; i < 3; ++i) {
    L S = staple_sum<G, T>(U, g, x, i, inv_a2);
    L Ui;
    load_link(Ui, U, i, s, V);
    A f = G::proj(G::mul(Ui, S));
    A e;
    load_alg(e, E + (int64_t)i * NG * V, s, V);
    const T kf = (T)(-c.dt / c.a[i]);
#pragma unroll
    for (int k = 0; k < NG; ++k) e.c[k] += kf * f.c[k];
    if (HOP && i == 2) {
      const int64_t sB = site_index(g, x.x, x.y, slotB(x.z, c.offB, g.nz));
      const int64_t sA = site_index(g, x.x, x.y, slotA(wrap_add(x.z, 1, g.nz), c.offA, g.nz));
      A rb, ra;
      load_alg(rb, rhoB, sB, V);
      load_alg(ra, rhoA, sA, V);
      A rbn = G::transport(Ui, rb);
      A ran = G::transport_inv(Ui, ra);
      store_alg(rbn, rhoB, sB, V);
      store_alg(ran, rhoA, sA, V);
      // dt * j_z = a_L (rho_A' - rho_B)
      const T al = (T)c.a[2];
#pragma unroll
      for (int k = 0; k < NG; ++k) e.c[k] += al * (ran.c[k] - rb.c[k]);
    }
    store_alg(e, E + (int64_t)i * NG * V, s, V);
    L Un = G::mul(G::expi(e, (T)(c.a[i] * c.dt)), Ui);
    store_link(Un, Unew, i, s, V);
  }
}

template <typename G, typename T>
void launch_leapfrog(const T* U, T* Unew, T* E, T* rhoA, T* rhoB, const Geom& g, const StepConst& c,
                     hipStream_t st) {
  const int bs = 256;
  const int64_t nb = (g.V + bs - 1) / bs;
  if (c.hop)
    hipLaunchKernelGGL((k_leapfrog<G, T, true>), dim3((unsigned)nb), dim3(bs), 0, st, U, Unew, E, rhoA, rhoB, g, c);
  else
    hipLaunchKernelGGL((k_leapfrog<G, T, false>), dim3((unsigned)nb), dim3(bs), 0, st, U, Unew, E, rhoA, rhoB, g, c);
}

template void launch_leapfrog<Su2<double>, double>(const double*, double*, double*, double*, double*, const Geom&, const StepConst&, hipStream_t);
template void launch_leapfrog<Su3<double>, double>(const double*, double*, double*, double*, double*, const Geom&, const StepConst&, hipStream_t);
template void launch_leapfrog<Su2<float>, float>(const float*, float*, float*, float*, float*, const Geom&, const StepConst&, hipStream_t);
template void launch_leapfrog<Su3<float>, float>(const float*, float*, float*, float*, float*, const Geom&, const StepConst&, hipStream_t);

}  // namespace gl
