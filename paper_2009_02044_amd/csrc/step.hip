// Leapfrog step with the CPIC charge hop (Sec. 3: eqs. lattice_1, lattice_2,
// plaquette, continuity and the nearest-grid-point transport rule).
//
// One thread owns one site x and its three links.  It forms the force terms
//   f_i = sum_{j != i} a_j^-2 P(U_{i,j}(x) + U_{i,-j}(x))
// plaquette by plaquette (stencil.h: plaquette_forces; a forward plaquette serves
// both of its directions), then for each direction updates
//   E_i += dt ( -(1/a_i) f_i + j_i ),   U_i' = exp(i a_i dt E_i) U_i,
// writing U' into the second link buffer (old links stay readable by the
// neighbours) and E in place.  On a hop step the z-link update also moves both
// charge populations one cell with parallel transport and adds the current that
// satisfies the continuity equation exactly:
//   B (+z): rho_B(x+z) <- U_z^dag(x) rho_B(x) U_z(x),     j_z(x) -= (a_L/dt) rho_B(x)
//   A (-z): rho_A(x)   <- U_z(x) rho_A(x+z) U_z^dag(x),   j_z(x) += (a_L/dt) rho_A'(x)
// With co-moving charge storage both rewrites are in place (one slot per thread).
#include "internal.h"
#include "stencil.h"
#include "reduce.h"

namespace gl {

template <typename R> __device__ __forceinline__ M3<double> to_double(const M3<R>& a) {
  M3<double> r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) { r.re[i][j] = (double)a.re[i][j]; r.im[i][j] = (double)a.im[i][j]; }
  return r;
}
template <typename R> __device__ __forceinline__ Q2<double> to_double(const Q2<R>& a) {
  Q2<double> r;
#pragma unroll
  for (int k = 0; k < 4; ++k) r.q[k] = (double)a.q[k];
  return r;
}

// Work-group size of the step kernel.
constexpr int LF_BS = 256;

// Observables gathered by an observing step (FP64): the E and B parts of T^{mu nu} at the
// integer time of the state the step starts from (E averaged over the two half steps,
// B from the forward plaquettes) and a non-finite flag (the Gauss-residual pass before the
// step measures the link unitarity).  The
// plaquette sums hand it each forward plaquette (plane<K>); the S_L terms are formed
// there, with E_i(t + dt/2) computed as the link update computes it, so that no
// projection stays live until the link update.
template <typename G, typename T> struct ObsAcc {
  double EL2 = 0.0, ET2 = 0.0, sl = 0.0;
  bool bad = false;
  const T* E;
  uint32_t s;
  int64_t Vp;
  StepConst c;
  double inv_a2[3];
  double* trs;
  // S_L = sum_a (Ebar_x^a P(U_xz)^a / (a_z a_x) + Ebar_y^a P(U_yz)^a / (a_y a_z)).  The real
  // traces of the forward plaquettes (for B^2) are parked in the work-group's LDS,
  // trs[K LF_BS + t], until the end of the step: carried in registers they would hold the
  // step at one wave per SIMD.
  template <int K>
  __device__ __forceinline__ void plane(const typename G::Alg& p, typename G::Real tr, const typename G::Alg& fi) {
    trs[K * LF_BS + threadIdx.x] = (double)tr;
    if constexpr (K > 0) {
      constexpr int i = K - 1;
      typename G::Alg eo;
      load_alg_own(eo, E, i, s, Vp);
      const double ai = c.a[i];
      const T kf = (T)(-c.dt / ai);
      double d = 0.0;
#pragma unroll
      for (int k = 0; k < G::NG; ++k) {
        const T en = fmx(kf, fi.c[k], eo.c[k]);
        d += 0.5 * ((double)eo.c[k] + (double)en) * (double)p.c[k];
      }
      sl += d / (c.a[2] * ai);
    }
  }
};

// Update of link (x, i) from the force term f_i of plaquette_forces (F_i = -f_i / a_i);
// the z-link thread also hops the charges.
template <typename G, typename T, bool HOP, bool OBS = false>
__device__ __forceinline__ void finish_link(const typename G::Link& Ui, const typename G::Alg& fi,
                                            T* __restrict__ Unew, T* __restrict__ E, T* __restrict__ rhoA,
                                            T* __restrict__ rhoB, const Geom& g, const StepConst& c, Site x,
                                            uint32_t s, int i, bool reunit, ObsAcc<G, T>* oa = nullptr) {
  using L = typename G::Link;
  using A = typename G::Alg;
  constexpr int NG = G::NG;
  const int64_t Vp = g.Vp;
  // i is a run-time value: select the spacing (no indexed local array)
  const double ai = i == 0 ? c.a[0] : (i == 1 ? c.a[1] : c.a[2]);
  A e;
  load_alg_own(e, E, i, s, Vp);
  A eo;
  if constexpr (OBS) eo = e;
  const T kf = (T)(-c.dt / ai);
#pragma unroll
  for (int k = 0; k < NG; ++k) e.c[k] = fmx(kf, fi.c[k], e.c[k]);
  if (HOP && c.hop && i == 2) {
    const uint32_t sB = site_index(g, x.x, x.y, slotB(x.z, c.offB, g.nz));
    const uint32_t sA = site_index(g, x.x, x.y, slotA(wrap_add(x.z, 1, g.nz), c.offA, g.nz));
    A rb, ra;
    load_alg_own(rb, rhoB, 0, sB, Vp);
    load_alg_own(ra, rhoA, 0, sA, Vp);
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
  if constexpr (OBS) {
    // E^2 averaged over the half steps
    const double e2 = 0.5 * (norm2(eo) + norm2(e));
    if (i == 2) oa->EL2 = e2; else oa->ET2 += e2;
#pragma unroll
    for (int k = 0; k < NG; ++k) oa->bad |= !isfinite((double)e.c[k]);
  }
  L Un = G::template expi_mul<true>(e, (T)(ai * c.dt), Ui);
  if (reunit) {
    // projection back onto SU(N) in double arithmetic
    using Gd = typename GroupOf<G::NC, double>::type;
    store_link(Gd::reunit(to_double(Un)), Unew, i, s, Vp);
  } else {
    store_link(Un, Unew, i, s, Vp);
  }
}

// The whole site update from plaquette forces.
template <typename G, typename T, bool HOP, bool XS, int OWN, bool OBS = false>
__device__ __forceinline__ void update_site(const T* __restrict__ U, T* __restrict__ Unew, T* __restrict__ E,
                                            T* __restrict__ rhoA, T* __restrict__ rhoB, const Geom& g,
                                            const StepConst& c, const double* inv_a2, Site x, uint32_t s,
                                            bool reunit, typename Vec16<T>::type* slot, uint32_t TB,
                                            ObsAcc<G, T>* oa = nullptr) {
  using L = typename G::Link;
  const GlobalLinks<T> fetch{U, g.Vp};
  const OwnLinks<G, T, OWN> own(fetch, s, slot, threadIdx.x, TB);
  typename G::Alg f[3];
  if constexpr (OBS) plaquette_forces<G, XS, true>(fetch, own, g, x, inv_a2, f, oa);
  else plaquette_forces<G, XS>(fetch, own, g, x, inv_a2, f);
#pragma unroll 1
  for (int i = 0; i < 3; ++i) {
    L Ui;
    own(Ui, i);
    typename G::Alg fi;
#pragma unroll
    for (int k = 0; k < G::NG; ++k) fi.c[k] = i == 0 ? f[0].c[k] : (i == 1 ? f[1].c[k] : f[2].c[k]);
    finish_link<G, T, HOP, OBS>(Ui, fi, Unew, E, rhoA, rhoB, g, c, x, s, i, reunit, oa);
  }
}

#ifndef GL_OWN64
#define GL_OWN64 OWN_LDS
#endif
#ifndef GL_OWN32
#define GL_OWN32 OWN_LDS
#endif
template <typename G, typename T> struct OwnMode {
  static constexpr int value = sizeof(T) == 8 ? GL_OWN64 : GL_OWN32;
};
// LDS for the own-link slots of a work-group of TB threads (one element when unused)
template <typename G, typename T, int TB> struct OwnLds {
  static constexpr int N = OwnMode<G, T>::value == OWN_LDS ? 3 * OwnSlot<G, T>::NCH * TB : 1;
};

#ifndef GL_LF_WAVES
#define GL_LF_WAVES 1
#endif
// One thread per site, the three directions in turn.  OBS: also gather the observables of the state the step starts from into the partial
// sums of this work-group (full work-groups only: every thread reaches the reduction).
// The observing variant is held to two waves per SIMD (its traces live in LDS, below).
// RU: the step also reunitarises the new links (in double arithmetic, before the store).
template <typename G, typename T, bool HOP, bool XS, bool OBS = false, bool RU = false>
__global__ void __launch_bounds__(LF_BS, OBS ? 2 : GL_LF_WAVES) k_leapfrog(const T* __restrict__ U, T* __restrict__ Unew,
                                                                 T* __restrict__ E, T* __restrict__ rhoA,
                                                                 T* __restrict__ rhoB, Geom g, StepConst c,
                                                                 ColMap m, double* __restrict__ partial = nullptr) {
  Site x;
  uint32_t s;
  __shared__ typename Vec16<T>::type slot[OwnLds<G, T, LF_BS>::N];
  if (!col_map_site(g, m, blockIdx.x, threadIdx.x, LF_BS, x, s)) return;
  const double inv_a2[3] = {1.0 / (c.a[0] * c.a[0]), 1.0 / (c.a[1] * c.a[1]), 1.0 / (c.a[2] * c.a[2])};
  if constexpr (!OBS) {
    update_site<G, T, HOP, XS, OwnMode<G, T>::value>(U, Unew, E, rhoA, rhoB, g, c, inv_a2, x, s, RU, slot, LF_BS);
  } else {
    __shared__ double trs[3 * LF_BS];
    ObsAcc<G, T> oa;
    oa.trs = trs;
    oa.E = E;
    oa.s = s;
    oa.Vp = g.Vp;
    oa.c = c;
#pragma unroll
    for (int k = 0; k < 3; ++k) oa.inv_a2[k] = inv_a2[k];
    update_site<G, T, HOP, XS, OwnMode<G, T>::value, true>(U, Unew, E, rhoA, rhoB, g, c, inv_a2, x, s, false, slot,
                                                           LF_BS, &oa);
    // B^2 = 4/(a_i a_j)^2 Re Tr(1 - U_ij) (U_{z,x} = U_{x,z}^dag has the same trace); each
    // thread reads back only its own trace slots
    const double nc = (double)G::NC;
    const double BL2 = 4.0 * inv_a2[0] * inv_a2[1] * (nc - trs[threadIdx.x]);
    double BT2 = 4.0 * inv_a2[0] * inv_a2[2] * (nc - trs[LF_BS + threadIdx.x]);
    BT2 += 4.0 * inv_a2[1] * inv_a2[2] * (nc - trs[2 * LF_BS + threadIdx.x]);
    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
    acc[Q_EPS] = 0.5 * (oa.EL2 + oa.ET2 + BL2 + BT2);
    acc[Q_PL] = 0.5 * (oa.ET2 + BT2 - oa.EL2 - BL2);
    acc[Q_PT] = 0.5 * (oa.EL2 + BL2);
    acc[Q_SL] = oa.sl;
    acc[Q_BAD] = (oa.bad || !isfinite(acc[Q_EPS])) ? 1.0 : 0.0;
    int zb;
    uint32_t slot;
    col_map_block(m, blockIdx.x, zb, slot);
    const unsigned mask = (1u << Q_EPS) | (1u << Q_PL) | (1u << Q_PT) | (1u << Q_SL) | (1u << Q_BAD);
    block_reduce_write<LF_BS, 1u << Q_BAD>(acc, mask, partial + ((int64_t)x.z * col_map_slots_per_layer(m) + slot) * NQ);
  }
}

template <typename G, typename T>
void launch_leapfrog(const T* U, T* Unew, T* E, T* rhoA, T* rhoB, const Geom& g, const StepConst& c,
                     bool reunit, hipStream_t st) {
  const int bs = LF_BS;
  const ColMap m = col_map(g, bs);
  const dim3 grid(col_map_blocks(g, m));
  // rows inside wavefronts: x neighbours from other lanes
  const bool xs = rows_in_wavefronts(g.nt);
  auto go = [&](auto kernel) { hipLaunchKernelGGL(kernel, grid, dim3(bs), 0, st, U, Unew, E, rhoA, rhoB, g, c, m, nullptr); };
  if (!reunit) {
    if (c.hop) xs ? go(k_leapfrog<G, T, true, true>) : go(k_leapfrog<G, T, true, false>);
    else xs ? go(k_leapfrog<G, T, false, true>) : go(k_leapfrog<G, T, false, false>);
  } else {
    if (c.hop) xs ? go(k_leapfrog<G, T, true, true, false, true>) : go(k_leapfrog<G, T, true, false, false, true>);
    else xs ? go(k_leapfrog<G, T, false, true, false, true>) : go(k_leapfrog<G, T, false, false, false, true>);
  }
}

// The observing step: the leapfrog step that also writes the energy slots of the
// observables of the state it starts from (FP64; nt a multiple of 64, so the column map
// has only full work-groups).  x neighbours come from adjacent lanes when a row lies in a
// wavefront (nt = 64), else from memory, as in the plain step.
template <typename G, typename T>
void launch_leapfrog_observe(const T* U, T* Unew, T* E, T* rhoA, T* rhoB, const Geom& g, const StepConst& c,
                             double* partial, hipStream_t st) {
  const int bs = LF_BS;
  const ColMap m = col_map(g, bs);
  const unsigned nbc = col_map_blocks(g, m);
  const bool xs = rows_in_wavefronts(g.nt);
  if (c.hop) {
    if (xs) hipLaunchKernelGGL((k_leapfrog<G, T, true, true, true>), dim3(nbc), dim3(bs), 0, st, U, Unew, E, rhoA,
                               rhoB, g, c, m, partial);
    else hipLaunchKernelGGL((k_leapfrog<G, T, true, false, true>), dim3(nbc), dim3(bs), 0, st, U, Unew, E, rhoA,
                            rhoB, g, c, m, partial);
  } else {
    if (xs) hipLaunchKernelGGL((k_leapfrog<G, T, false, true, true>), dim3(nbc), dim3(bs), 0, st, U, Unew, E, rhoA,
                               rhoB, g, c, m, partial);
    else hipLaunchKernelGGL((k_leapfrog<G, T, false, false, true>), dim3(nbc), dim3(bs), 0, st, U, Unew, E, rhoA,
                            rhoB, g, c, m, partial);
  }
}
template void launch_leapfrog_observe<Su3<double>, double>(const double*, double*, double*, double*, double*,
                                                          const Geom&, const StepConst&, double*, hipStream_t);
template void launch_leapfrog_observe<Su2<double>, double>(const double*, double*, double*, double*, double*,
                                                          const Geom&, const StepConst&, double*, hipStream_t);

// ---- batched form: many events of different sizes in one launch --------------

// Work item = `bs` consecutive sites of one event: one work-group per item, or persistent
// work-groups that loop over the items.  The step number comes
// from device memory so that a captured graph of several steps replays correctly:
// parity of the link buffers, hop flag and charge offsets all follow from it.
GL_HD int64_t hop_count_dev(int64_t s, int64_t p, int64_t q) { return ((2 * s + 1) * p + q) / (2 * q); }

// Per-step values of the batch, from the device step counter.
struct BatchStep {
  int64_t st, S0;
  bool hop, reunit;
  double inv_a2[3];
};
__device__ __forceinline__ BatchStep batch_step_of(const BatchConst& bc, const int64_t* __restrict__ ctr) {
  BatchStep b;
  b.st = ctr[0];
  const int64_t S1 = hop_count_dev(b.st, bc.hop_p, bc.hop_q);
  b.S0 = hop_count_dev(b.st - 1, bc.hop_p, bc.hop_q);
  b.hop = S1 > b.S0;
  b.reunit = bc.reunit_every > 0 && ((b.st + 1) % bc.reunit_every) == 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) b.inv_a2[k] = 1.0 / (bc.a[k] * bc.a[k]);
  return b;
}

// One work item: blockDim.x consecutive sites of one event.
template <typename G, typename T>
__device__ __forceinline__ void batch_item(char* __restrict__ pool, const EventDesc* __restrict__ ev,
                                           const uint32_t* __restrict__ item_event, const BatchConst& bc,
                                           const BatchStep& b, uint32_t item, typename Vec16<T>::type* slot) {
  const EventDesc d = ev[item_event[item]];
  const uint32_t s = (item - d.item0) * blockDim.x + threadIdx.x;
  if (s >= (uint32_t)d.g.V) return;
  StepConst c;
  c.a[0] = bc.a[0]; c.a[1] = bc.a[1]; c.a[2] = bc.a[2];
  c.dt = bc.dt;
  c.hop = b.hop ? 1 : 0;
  const int64_t off = (d.off0 + (b.S0 - d.hops0)) % d.g.nz;
  c.offA = (int)off;
  c.offB = (int)off;
  c.scheme = 0;
  const bool odd = (b.st & 1) != 0;
  const T* U = (const T*)(pool + (odd ? d.Uodd : d.Ueven));
  T* Un = (T*)(pool + (odd ? d.Ueven : d.Uodd));
  Site x;
  x.x = (int)(s % (uint32_t)d.g.nt);
  x.y = (int)((s / (uint32_t)d.g.nt) % (uint32_t)d.g.nt);
  x.z = (int)(s / (uint32_t)d.g.layer);
  // item = 64-aligned sites of one event: rows lie in wavefronts when nt divides 64
  constexpr int K = OwnMode<G, T>::value;
  T *E = (T*)(pool + d.E), *rA = (T*)(pool + d.rhoA), *rB = (T*)(pool + d.rhoB);
  const uint32_t TB = blockDim.x;
  const Geom g = d.g;
  // the hop branch inside is uniform over the launch (HOP = true only enables it)
  if (rows_in_wavefronts(g.nt))
    update_site<G, T, true, true, K>(U, Un, E, rA, rB, g, c, b.inv_a2, x, s, b.reunit, slot, TB);
  else
    update_site<G, T, true, false, K>(U, Un, E, rA, rB, g, c, b.inv_a2, x, s, b.reunit, slot, TB);
}

// Items are dealt to the XCDs in chunks of 64 (xcd_chunk_remap): 2.5% faster than one by one
// on a mix of 64 events, which keeps the XCDs' shares of the events balanced.
constexpr uint32_t BATCH_XCD_CHUNK = 64;

// Persistent form: `grid` work-groups loop over the items (a grid that is a multiple of 8
// keeps each work-group's indices on its own XCD).
template <typename G, typename T>
__global__ void __launch_bounds__(256) k_batch_step(char* __restrict__ pool, const EventDesc* __restrict__ ev,
                                                    const uint32_t* __restrict__ item_event, BatchConst bc,
                                                    const int64_t* __restrict__ ctr) {
  const BatchStep b = batch_step_of(bc, ctr);
  __shared__ typename Vec16<T>::type slot[OwnLds<G, T, 256>::N];
  for (uint32_t v = blockIdx.x; v < bc.items; v += gridDim.x)
    batch_item<G, T>(pool, ev, item_event, bc, b, xcd_chunk_remap<BATCH_XCD_CHUNK>(v, bc.items), slot);
}

// One work-group per item.  Without the loop the FP32 kernel fits 128 registers and runs at
// four waves per SIMD (the loop costs it ~23 registers and a wave).
template <typename G, typename T>
__global__ void __launch_bounds__(256, sizeof(T) == 4 ? 4 : 1)
    k_batch_step_flat(char* __restrict__ pool, const EventDesc* __restrict__ ev,
                      const uint32_t* __restrict__ item_event, BatchConst bc, const int64_t* __restrict__ ctr) {
  const BatchStep b = batch_step_of(bc, ctr);
  __shared__ typename Vec16<T>::type slot[OwnLds<G, T, 256>::N];
  if (blockIdx.x < bc.items)
    batch_item<G, T>(pool, ev, item_event, bc, b, xcd_chunk_remap<BATCH_XCD_CHUNK>(blockIdx.x, bc.items), slot);
}

// advance the device step counter (one lane writes)
__global__ void k_batch_tick(int64_t* ctr) {
  if (threadIdx.x == 0) {
    const int64_t v = ctr[0];
    ctr[threadIdx.x] = v + 1;
  }
}

template <typename G, typename T>
void launch_batch_step(char* pool, const EventDesc* ev, const uint32_t* item_event, const BatchConst& bc,
                       const int64_t* ctr, int grid, int bs, hipStream_t st) {
  if (grid > 0)
    hipLaunchKernelGGL((k_batch_step<G, T>), dim3((unsigned)grid), dim3((unsigned)bs), 0, st, pool, ev, item_event, bc,
                       ctr);
  else
    hipLaunchKernelGGL((k_batch_step_flat<G, T>), dim3(bc.items), dim3((unsigned)bs), 0, st, pool, ev, item_event,
                       bc, ctr);
}
void launch_batch_tick(int64_t* ctr, hipStream_t st) { hipLaunchKernelGGL(k_batch_tick, dim3(1), dim3(64), 0, st, ctr); }

template void launch_batch_step<Su2<double>, double>(char*, const EventDesc*, const uint32_t*, const BatchConst&, const int64_t*, int, int, hipStream_t);
template void launch_batch_step<Su3<double>, double>(char*, const EventDesc*, const uint32_t*, const BatchConst&, const int64_t*, int, int, hipStream_t);
template void launch_batch_step<Su2<float>, float>(char*, const EventDesc*, const uint32_t*, const BatchConst&, const int64_t*, int, int, hipStream_t);
template void launch_batch_step<Su3<float>, float>(char*, const EventDesc*, const uint32_t*, const BatchConst&, const int64_t*, int, int, hipStream_t);

template void launch_leapfrog<Su2<double>, double>(const double*, double*, double*, double*, double*, const Geom&, const StepConst&, bool, hipStream_t);
template void launch_leapfrog<Su3<double>, double>(const double*, double*, double*, double*, double*, const Geom&, const StepConst&, bool, hipStream_t);
template void launch_leapfrog<Su2<float>, float>(const float*, float*, float*, float*, float*, const Geom&, const StepConst&, bool, hipStream_t);
template void launch_leapfrog<Su3<float>, float>(const float*, float*, float*, float*, float*, const Geom&, const StepConst&, bool, hipStream_t);

}  // namespace gl
