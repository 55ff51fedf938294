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

// Update of link (x, i): staples, E, CPIC hop (z links on hop steps), exp, new link.
// fetch(l, d, s) supplies the links at time t (from the work-group's LDS tile or memory).
template <typename G, typename T, bool HOP, typename F>
__device__ __forceinline__ void update_link(const F& fetch, T* __restrict__ Unew, T* __restrict__ E,
                                            T* __restrict__ rhoA, T* __restrict__ rhoB, const Geom& g,
                                            const StepConst& c, const double* inv_a2, Site x, uint32_t s, int i,
                                            bool reunit = false) {
  using L = typename G::Link;
  using A = typename G::Alg;
  constexpr int NG = G::NG;
  const int64_t Vp = g.Vp;
  const double w1 = inv_a2[other_lo(i)], w2 = inv_a2[other_hi(i)];
  L S = staple_sum_scaled_f<G>(fetch, g, x, i, (T)(w1 / w2));
  L Ui;
  fetch(Ui, i, s);
  A f = G::proj_mul(Ui, S);
  A e;
  load_alg(e, E, i, s, Vp);
  const T kf = (T)(-c.dt / c.a[i] * w2);
#pragma unroll
  for (int k = 0; k < NG; ++k) e.c[k] += kf * f.c[k];
  if (HOP && i == 2) {
    const uint32_t sB = site_index(g, x.x, x.y, slotB(x.z, c.offB, g.nz));
    const uint32_t sA = site_index(g, x.x, x.y, slotA(wrap_add(x.z, 1, g.nz), c.offA, g.nz));
    A rb, ra;
    load_alg(rb, rhoB, 0, sB, Vp);
    load_alg(ra, rhoA, 0, sA, Vp);
    A rbn = G::transport(Ui, rb);
    A ran = G::transport_inv(Ui, ra);
    store_alg(rbn, rhoB, 0, sB, Vp);
    store_alg(ran, rhoA, 0, sA, Vp);
    // dt * j_z = a_L (rho_A' - rho_B)
    const T al = (T)c.a[2];
#pragma unroll
    for (int k = 0; k < NG; ++k) e.c[k] += al * (ran.c[k] - rb.c[k]);
  }
  store_alg(e, E, i, s, Vp);
  // rows 0 and 1 are all that the link storage (and the reunitarisation) use
  L Un = G::template expi_mul<true>(e, (T)(c.a[i] * c.dt), Ui);
  if (reunit) {
    // projection back onto SU(N) in double arithmetic
    using Gd = typename GroupOf<G::NC, double>::type;
    typename Gd::Link ud;
    const T* un = reinterpret_cast<const T*>(&Un);
    double* dd = reinterpret_cast<double*>(&ud);
    for (int k = 0; k < (int)(sizeof(L) / sizeof(T)); ++k) dd[k] = (double)un[k];
    store_link(Gd::reunit(ud), Unew, i, s, Vp);
  } else {
    store_link(Un, Unew, i, s, Vp);
  }
}

#ifndef GL_LF_WAVES
#define GL_LF_WAVES 1
#endif
// One thread per site, the three directions in turn.
constexpr int LF_BS = 256;
template <typename G, typename T, bool HOP>
__global__ void __launch_bounds__(LF_BS, GL_LF_WAVES) k_leapfrog(const T* __restrict__ U, T* __restrict__ Unew,
                                                                 T* __restrict__ E, T* __restrict__ rhoA,
                                                                 T* __restrict__ rhoB, Geom g, StepConst c,
                                                                 ColMap m) {
  Site x;
  uint32_t s;
  if (!col_map_site(g, m, blockIdx.x, threadIdx.x, LF_BS, x, s)) return;
  const GlobalLinks<T> f{U, g.Vp};
  const double inv_a2[3] = {1.0 / (c.a[0] * c.a[0]), 1.0 / (c.a[1] * c.a[1]), 1.0 / (c.a[2] * c.a[2])};
#pragma unroll 1
  for (int i = 0; i < 3; ++i) update_link<G, T, HOP>(f, Unew, E, rhoA, rhoB, g, c, inv_a2, x, s, i);
}

template <typename G, typename T>
void launch_leapfrog(const T* U, T* Unew, T* E, T* rhoA, T* rhoB, const Geom& g, const StepConst& c,
                     hipStream_t st) {
  const int bs = LF_BS;
  const ColMap m = col_map(g, bs);
  const unsigned nbc = col_map_blocks(g, m);
  if (c.hop)
    hipLaunchKernelGGL((k_leapfrog<G, T, true>), dim3(nbc), dim3(bs), 0, st, U, Unew, E, rhoA, rhoB, g, c, m);
  else
    hipLaunchKernelGGL((k_leapfrog<G, T, false>), dim3(nbc), dim3(bs), 0, st, U, Unew, E, rhoA, rhoB, g, c, m);
}

// ---- batched form: many events of different sizes in one launch --------------
// Work item = `bs` consecutive sites of one event; workgroups loop over the items
// (persistent when the grid is smaller than the item count).  The step number comes
// from device memory so that a captured graph of several steps replays correctly:
// parity of the link buffers, hop flag and charge offsets all follow from it.
GL_HD int64_t hop_count_dev(int64_t s, int64_t p, int64_t q) { return ((2 * s + 1) * p + q) / (2 * q); }

template <typename G, typename T>
__global__ void __launch_bounds__(256) k_batch_step(const EventDesc* __restrict__ ev,
                                                    const uint32_t* __restrict__ item_event, BatchConst bc,
                                                    const int64_t* __restrict__ ctr) {
  const int64_t st = ctr[0];
  const int64_t S1 = hop_count_dev(st, bc.hop_p, bc.hop_q), S0 = hop_count_dev(st - 1, bc.hop_p, bc.hop_q);
  const bool hop = S1 > S0;
  const bool reunit = bc.reunit_every > 0 && ((st + 1) % bc.reunit_every) == 0;
  const double inv_a2[3] = {1.0 / (bc.a[0] * bc.a[0]), 1.0 / (bc.a[1] * bc.a[1]), 1.0 / (bc.a[2] * bc.a[2])};
  for (uint32_t item = blockIdx.x; item < bc.items; item += gridDim.x) {
    const EventDesc d = ev[item_event[item]];
    const uint32_t s = (item - d.item0) * blockDim.x + threadIdx.x;
    if (s >= (uint32_t)d.g.V) continue;
    StepConst c;
    c.a[0] = bc.a[0]; c.a[1] = bc.a[1]; c.a[2] = bc.a[2];
    c.dt = bc.dt;
    c.hop = hop ? 1 : 0;
    const int64_t off = (d.off0 + (S0 - d.hops0)) % d.g.nz;
    c.offA = (int)off;
    c.offB = (int)off;
    c.scheme = 0;
    const bool odd = (st & 1) != 0;
    const T* U = (const T*)(odd ? d.Uodd : d.Ueven);
    T* Un = (T*)(odd ? d.Ueven : d.Uodd);
    Site x;
    x.x = (int)(s % (uint32_t)d.g.nt);
    x.y = (int)((s / (uint32_t)d.g.nt) % (uint32_t)d.g.nt);
    x.z = (int)(s / (uint32_t)d.g.layer);
    const GlobalLinks<T> f{U, d.g.Vp};
#pragma unroll 1
    for (int i = 0; i < 3; ++i) {
      if (hop)
        update_link<G, T, true>(f, Un, (T*)d.E, (T*)d.rhoA, (T*)d.rhoB, d.g, c, inv_a2, x, s, i, reunit);
      else
        update_link<G, T, false>(f, Un, (T*)d.E, (T*)d.rhoA, (T*)d.rhoB, d.g, c, inv_a2, x, s, i, reunit);
    }
  }
}

// advance the device step counter (one lane writes)
__global__ void k_batch_tick(int64_t* ctr) {
  if (threadIdx.x == 0) {
    const int64_t v = ctr[0];
    ctr[threadIdx.x] = v + 1;
  }
}

template <typename G, typename T>
void launch_batch_step(const EventDesc* ev, const uint32_t* item_event, const BatchConst& bc, const int64_t* ctr,
                       int grid, int bs, hipStream_t st) {
  hipLaunchKernelGGL((k_batch_step<G, T>), dim3((unsigned)grid), dim3((unsigned)bs), 0, st, ev, item_event, bc, ctr);
}
void launch_batch_tick(int64_t* ctr, hipStream_t st) { hipLaunchKernelGGL(k_batch_tick, dim3(1), dim3(64), 0, st, ctr); }

template void launch_batch_step<Su2<double>, double>(const EventDesc*, const uint32_t*, const BatchConst&, const int64_t*, int, int, hipStream_t);
template void launch_batch_step<Su3<double>, double>(const EventDesc*, const uint32_t*, const BatchConst&, const int64_t*, int, int, hipStream_t);
template void launch_batch_step<Su2<float>, float>(const EventDesc*, const uint32_t*, const BatchConst&, const int64_t*, int, int, hipStream_t);
template void launch_batch_step<Su3<float>, float>(const EventDesc*, const uint32_t*, const BatchConst&, const int64_t*, int, int, hipStream_t);

template void launch_leapfrog<Su2<double>, double>(const double*, double*, double*, double*, double*, const Geom&, const StepConst&, hipStream_t);
template void launch_leapfrog<Su3<double>, double>(const double*, double*, double*, double*, double*, const Geom&, const StepConst&, hipStream_t);
template void launch_leapfrog<Su2<float>, float>(const float*, float*, float*, float*, float*, const Geom&, const StepConst&, hipStream_t);
template void launch_leapfrog<Su3<float>, float>(const float*, float*, float*, float*, float*, const Geom&, const StepConst&, hipStream_t);

}  // namespace gl
