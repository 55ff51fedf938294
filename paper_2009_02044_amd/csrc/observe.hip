// Observables (Sec. 4: <T^{mu nu}> components and eq. pT_eL; Sec. 3: eq. gauss),
// the CPIC current of the next step, and FP64 reunitarisation of the links.
//
// At integer time t (state U(t), E(t - dt/2), rho(t - dt/2)) every thread recomputes
// the leapfrog E update of its site in double precision without applying it (or, for the
// semi-implicit scheme, reads E(t + dt/2) from the converged solve of the step that
// follows, En), then forms
//   E_i^2 = (|E_i(t-dt/2)|^2 + |E_i(t+dt/2)|^2)/2,
//   B_ij^2 = 4/(a_i a_j)^2 Re Tr(1 - U_{i,j}),  F_ij^a = proj(U_{i,j})^a / (a_i a_j),
//   eps = (E^2 + B^2)/2, p_T = (E_L^2 + B_L^2)/2, p_L = (E_T^2 + B_T^2 - E_L^2 - B_L^2)/2,
//   S_L = -sum_a (Ebar_x^a F_zx^a - Ebar_y^a F_yz^a),  Ebar = (E(t-dt/2) + E(t+dt/2))/2,
// (E = d_t A is minus the physical field, hence the sign of S_L), the Gauss residual
//   G(x) = sum_i [E_i(x) - U_i^dag(x-i) E_i(x-i) U_i(x-i)]/a_i - rho(x),
// link unitarity and a non-finite count.  A block covers part of one z layer; its
// partial sums land in a fixed slot and a single-block pass adds them in a fixed
// order, so results are bitwise reproducible.
#include <mutex>
#include <type_traits>
#include "internal.h"
#include "stencil.h"
#include "reduce.h"

namespace gl {

constexpr int OBS_BS = 256;
#ifndef GL_OBS_OWN
#define GL_OBS_OWN OWN_LDS
#endif

// one site per thread: the blocks of a layer cover it exactly once
static int obs_blocks_per_layer(const Geom& g) { return (int)((g.layer + OBS_BS - 1) / OBS_BS); }
size_t observe_partial_doubles(const Geom& g) {
  return (size_t)obs_blocks_per_layer(g) * g.nz * NQ;
}


// Plaquette observer of this pass: the S_L terms are formed where the (x, z) and (y, z)
// plaquettes are (f_x and f_y are complete there, see plaquette_forces), with
// E(t + dt/2) = E(t - dt/2) - dt f_i / a_i (leapfrog) or read from En (semi-implicit);
// the real traces (for B^2) are parked in LDS, trs[K OBS_BS + t], until the end.  Carrying
// the projections and traces in registers held the pass at one wave per SIMD.  HAS_EN is a
// template parameter: a run-time choice between the two sources of E(t + dt/2) made the
// compiler spill several hundred registers (a 3x slower pass).
template <typename G, typename T, bool HAS_EN> struct PassObs {
  const T* E;
  const T* En;
  uint32_t s;
  int64_t Vp;
  StepConst c;
  double* trs;
  double sl = 0.0;
  template <int K>
  __device__ __forceinline__ void plane(const typename G::Alg& p, typename G::Real tr, const typename G::Alg& fi) {
    trs[K * OBS_BS + threadIdx.x] = (double)tr;
    if constexpr (K > 0) {
      constexpr int i = K - 1;
      typename G::Alg eo, enx;
      load_alg(eo, E, i, s, Vp);
      if constexpr (HAS_EN) load_alg(enx, En, i, s, Vp);
      const double ai = c.a[i];
      double d = 0.0;
#pragma unroll
      for (int k = 0; k < G::NG; ++k) {
        double en;
        if constexpr (HAS_EN) en = (double)enx.c[k];
        else en = eo.c[k] - c.dt / ai * fi.c[k];
        d += 0.5 * (eo.c[k] + en) * p.c[k];
      }
      sl += d / (c.a[2] * ai);
    }
  }
};

// Links stored in FP32 are unitary only to the rounding of their stored rows (~1e-7), while
// 1 - Re Tr U_ij / N_c of a plaquette, which gives B^2, is small: read as stored they bias
// B^2 (and so eps, p_L, p_T) by ~1e-4 relative.  The pass therefore measures an FP32 state on
// its links projected onto SU(N) in double precision, every link as it is read; the unitarity
// observable reads the stored links.
// The projection of a link onto SU(N): Gram-Schmidt of its two stored rows and the third row
// rebuilt as for every load.  The reciprocal square roots come from the hardware estimate
// refined by two Newton steps y <- y (3 - n y^2) / 2 (each doubles the correct bits), without
// the division and square root of 1 / sqrt(n) and without a branch.
__device__ __forceinline__ double inv_sqrt_near1(double n) {
  double y = __builtin_amdgcn_rsq(n);
  y = y * (1.5 - 0.5 * n * y * y);
  return y * (1.5 - 0.5 * n * y * y);
}
__device__ __forceinline__ void project_near_unitary(M3<double>& r) {
  double n0 = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) n0 += r.re[0][k] * r.re[0][k] + r.im[0][k] * r.im[0][k];
  const double s0 = inv_sqrt_near1(n0);
#pragma unroll
  for (int k = 0; k < 3; ++k) { r.re[0][k] *= s0; r.im[0][k] *= s0; }
  double pr = 0.0, pi = 0.0;   // r0^dag r1
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    pr += r.re[0][k] * r.re[1][k] + r.im[0][k] * r.im[1][k];
    pi += r.re[0][k] * r.im[1][k] - r.im[0][k] * r.re[1][k];
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    r.re[1][k] -= pr * r.re[0][k] - pi * r.im[0][k];
    r.im[1][k] -= pr * r.im[0][k] + pi * r.re[0][k];
  }
  double n1 = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) n1 += r.re[1][k] * r.re[1][k] + r.im[1][k] * r.im[1][k];
  const double s1 = inv_sqrt_near1(n1);
#pragma unroll
  for (int k = 0; k < 3; ++k) { r.re[1][k] *= s1; r.im[1][k] *= s1; }
  complete_row2(r);
}
__device__ __forceinline__ void project_near_unitary(Q2<double>& q) {
  double n = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) n += q.q[k] * q.q[k];
  const double s = inv_sqrt_near1(n);
#pragma unroll
  for (int k = 0; k < 4; ++k) q.q[k] *= s;
}
// the stored reals of a link (rows 0 and 1, or the quaternion), the layout link_from_stored reads
__device__ __forceinline__ void link_to_stored(const M3<double>& l, double (&v)[SU3_STORED]) {
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      v[2 * (3 * r + k)] = l.re[r][k];
      v[2 * (3 * r + k) + 1] = l.im[r][k];
    }
}
__device__ __forceinline__ void link_to_stored(const Q2<double>& l, double (&v)[4]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = l.q[k];
}

// The site's own links for an FP32 state: loaded once, projected once, their two rows kept in
// double precision in a per-thread LDS slot (chunk q of direction d of thread t at
// [(d NCH + q) OBS_BS + t]) and the link rebuilt from there at every use.
template <typename G> struct OwnProjLds {
  static constexpr int W = StoredWidth<typename G::Link>::value;   // 12 or 4 doubles
  static constexpr int NCH = W / 2;                                // 16-byte chunks
  double2* lds;
  uint32_t t;
  template <typename T>
  __device__ __forceinline__ OwnProjLds(const GlobalLinks<T>& f, uint32_t s, double2* lds_, uint32_t t_)
      : lds(lds_), t(t_) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      typename G::Link l;
      f(l, d, s);
      project_near_unitary(l);
      double v[W];
      link_to_stored(l, v);
#pragma unroll
      for (int q = 0; q < NCH; ++q) lds[(d * NCH + q) * OBS_BS + t] = make_double2(v[2 * q], v[2 * q + 1]);
    }
  }
  __device__ __forceinline__ void operator()(typename G::Link& l, int d) const {
    uint32_t tt = t;
    asm volatile("" : "+v"(tt));
    double v[W];
#pragma unroll
    for (int q = 0; q < NCH; ++q) {
      const double2 x = lds[(d * NCH + q) * OBS_BS + tt];
      v[2 * q] = x.x;
      v[2 * q + 1] = x.y;
    }
    link_from_stored(l, v);
  }
};
template <typename G, typename T> struct ProjLinks {
  GlobalLinks<T> f;
  template <typename L> __device__ __forceinline__ void operator()(L& l, int d, uint32_t s) const {
    f(l, d, s);
    if constexpr (sizeof(T) == 4) project_near_unitary(l);
  }
};

template <typename G, typename T, bool XS, bool HAS_EN>
__global__ void __launch_bounds__(OBS_BS, 2) k_observe(const T* __restrict__ U, const T* __restrict__ E,
                                                    const T* __restrict__ rhoA, const T* __restrict__ rhoB,
                                                    const T* __restrict__ En, Geom g, StepConst c,
                                                    double* __restrict__ partial) {
  using L = typename G::Link;   // double precision group
  using A = typename G::Alg;
  constexpr int NG = G::NG;
  const int64_t Vp = g.Vp;
  const int z = blockIdx.y;
  const int nbx = gridDim.x;
  const double inv_a2[3] = {1.0 / (c.a[0] * c.a[0]), 1.0 / (c.a[1] * c.a[1]), 1.0 / (c.a[2] * c.a[2])};
  // own-link slots: the stored chunks (FP64 state) or the projected rows in double (FP32 state)
  constexpr bool PROJ = sizeof(T) == 4;
  constexpr int SLOT_BYTES = PROJ ? 3 * OwnProjLds<G>::NCH * OBS_BS * 16 : 3 * OwnSlot<G, T>::NCH * OBS_BS * 16;
  __shared__ double2 slot_mem[SLOT_BYTES / 16];
  __shared__ double trs[3 * OBS_BS];
  const GlobalLinks<T> fetch{U, Vp};
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
  // blocks start at multiples of 64 sites of the layer, so rows stay whole for XS
  const int64_t t = (int64_t)blockIdx.x * OBS_BS + threadIdx.x;
  if (t < g.layer) {
    const uint32_t s = (uint32_t)((int64_t)z * g.layer + t);
    Site x;
    x.x = (int)(t % g.nt);
    x.y = (int)(t / g.nt);
    x.z = z;
    // force terms of the E update, and the forward plaquettes, in double precision
    using OwnRaw = OwnLinks<G, T, GL_OBS_OWN>;
    using Own = std::conditional_t<PROJ, OwnProjLds<G>, OwnRaw>;
    auto own = [&]() -> Own {
      if constexpr (PROJ) return Own(fetch, s, slot_mem, threadIdx.x);
      else return Own(fetch, s, (typename Vec16<T>::type*)slot_mem, threadIdx.x, OBS_BS);
    }();
    A f[3];
    PassObs<G, T, HAS_EN> ob;
    ob.E = E;
    ob.En = En;
    ob.s = s;
    ob.Vp = Vp;
    ob.c = c;
    ob.trs = trs;
    const ProjLinks<G, T> pfetch{fetch};
    plaquette_forces<G, XS, true>(pfetch, own, g, x, inv_a2, f, &ob);
    double e2[3];
    bool bad = false;
    // one direction at a time (i is a run-time value: members are selected, not indexed)
#pragma unroll 1
    for (int i = 0; i < 3; ++i) {
      const double ai = i == 0 ? c.a[0] : (i == 1 ? c.a[1] : c.a[2]);
      A eo, en;
      load_alg(eo, E, i, s, Vp);
      if constexpr (HAS_EN) {
        // semi-implicit scheme: E(t + dt/2) of the converged solve (the current included)
        load_alg(en, En, i, s, Vp);
      } else {
        for (int k = 0; k < NG; ++k) {
          const double fk = i == 0 ? f[0].c[k] : (i == 1 ? f[1].c[k] : f[2].c[k]);
          en.c[k] = eo.c[k] - c.dt / ai * fk;
        }
      }
      L Ui;   // the stored link (the unitarity observable reads it as stored)
      fetch(Ui, i, s);
      if (!HAS_EN && c.hop && i == 2) {
        A rb, ra;
        load_alg(rb, rhoB, 0, site_index(g, x.x, x.y, slotB(z, c.offB, g.nz)), Vp);
        load_alg(ra, rhoA, 0, site_index(g, x.x, x.y, slotA(wrap_add(z, 1, g.nz), c.offA, g.nz)), Vp);
        A ran = G::transport_inv(Ui, ra);
        for (int k = 0; k < NG; ++k) en.c[k] += c.a[2] * (ran.c[k] - rb.c[k]);
      }
      for (int k = 0; k < NG; ++k) bad |= !isfinite(en.c[k]);
      const double ei = 0.5 * (norm2(eo) + norm2(en));
      e2[0] = i == 0 ? ei : e2[0];
      e2[1] = i == 1 ? ei : e2[1];
      e2[2] = i == 2 ? ei : e2[2];
      double uv = G::unit_violation(Ui);
      bad |= !isfinite(uv);
      acc[7] = fmax(acc[7], uv);
    }
    // B^2 from the forward plaquettes U_{x,y}, U_{y,z} and U_{z,x} = U_{x,z}^dag (same
    // real trace); F_yz = P(U_{y,z}), F_zx = P(U_{z,x}) = -P(U_{x,z})
    const double nc = (double)G::NC;
    const double bxy = 4.0 * inv_a2[0] * inv_a2[1] * (nc - trs[threadIdx.x]);
    const double bzx = 4.0 * inv_a2[2] * inv_a2[0] * (nc - trs[OBS_BS + threadIdx.x]);
    const double byz = 4.0 * inv_a2[1] * inv_a2[2] * (nc - trs[2 * OBS_BS + threadIdx.x]);
    const double sl = ob.sl;
    const double EL2 = e2[2], ET2 = e2[0] + e2[1], BL2 = bxy, BT2 = byz + bzx;
    acc[0] += 0.5 * (EL2 + ET2 + BL2 + BT2);
    acc[1] += 0.5 * (ET2 + BT2 - EL2 - BL2);
    acc[2] += 0.5 * (EL2 + BL2);
    acc[3] += sl;
    // Gauss residual at (U(t), E(t - dt/2), rho(t - dt/2))
    A G_, r, rb;
    load_alg(r, rhoA, 0, site_index(g, x.x, x.y, slotA(z, c.offA, g.nz)), Vp);
    load_alg(rb, rhoB, 0, site_index(g, x.x, x.y, slotB(z, c.offB, g.nz)), Vp);
    for (int k = 0; k < NG; ++k) { r.c[k] += rb.c[k]; G_.c[k] = -r.c[k]; }
#pragma unroll 1
    for (int i = 0; i < 3; ++i) {
      const double ai = i == 0 ? c.a[0] : (i == 1 ? c.a[1] : c.a[2]);
      Site xm = shifted(g, x, i, -1);
      const int64_t sm = idx(g, xm);
      L Um;
      load_link(Um, U, i, sm, Vp);
      A eh, em;
      load_alg(eh, E, i, s, Vp);
      load_alg(em, E, i, sm, Vp);
      A tr = G::transport(Um, em);
      for (int k = 0; k < NG; ++k) G_.c[k] += (eh.c[k] - tr.c[k]) / ai;
    }
    acc[4] += norm2(G_);
    acc[5] += norm2(r);
    double gm = 0.0;
    for (int k = 0; k < NG; ++k) gm = fmax(gm, fabs(G_.c[k]));
    acc[6] = fmax(acc[6], gm);
    bad |= !isfinite(acc[0]) || !isfinite(acc[4]);
    acc[8] += bad ? 1.0 : 0.0;
  }
  block_reduce_write<OBS_BS>(acc, Q_ALL, partial + ((int64_t)z * nbx + blockIdx.x) * NQ);
}

// Gauss residual, |rho|, link unitarity and the non-finite count over the step kernel's
// work-groups (column map), for the observing step: it runs before that step, which then
// adds the energy slots to the same partial sums.  G(x) = sum_i [E_i(x) - U_i^dag(x-i)
// E_i(x-i) U_i(x-i)]/a_i - rho(x) at (U(t), E(t - dt/2), rho(t - dt/2)).  Every link U_i(y)
// is read here exactly once, as U_i(x - i) of x = y + i, so the unitarity maximum over these
// reads is the maximum over all links (kept out of the step kernel, whose registers are at
// their limit).  Partial slot of block b: z nbx + its slot.
template <typename G, typename T>
__global__ void __launch_bounds__(256) k_obs_gauss(const T* __restrict__ U, const T* __restrict__ E,
                                                   const T* __restrict__ rhoA, const T* __restrict__ rhoB,
                                                   Geom g, StepConst c, ColMap m, double* __restrict__ partial,
                                                   int nbx) {
  using L = typename G::Link;
  using A = typename G::Alg;
  constexpr int NG = G::NG;
  const int64_t Vp = g.Vp;
  Site x;
  uint32_t s;
  const bool has = col_map_site(g, m, blockIdx.x, threadIdx.x, blockDim.x, x, s);
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
  bool bad = false;
  if (has) {
    A G_, r, rb;
    load_alg(r, rhoA, 0, site_index(g, x.x, x.y, slotA(x.z, c.offA, g.nz)), Vp);
    load_alg(rb, rhoB, 0, site_index(g, x.x, x.y, slotB(x.z, c.offB, g.nz)), Vp);
    for (int k = 0; k < NG; ++k) { r.c[k] += rb.c[k]; G_.c[k] = -r.c[k]; }
#pragma unroll 1
    for (int i = 0; i < 3; ++i) {
      const double ai = i == 0 ? c.a[0] : (i == 1 ? c.a[1] : c.a[2]);
      const uint32_t sm = idx(g, shifted(g, x, i, -1));
      L Um;
      load_link(Um, U, i, sm, Vp);
      const double uv = G::unit_violation(Um);
      acc[Q_UNIT] = fmax(acc[Q_UNIT], uv);
      bad |= !isfinite(uv);
      A eh, em;
      load_alg(eh, E, i, s, Vp);
      load_alg(em, E, i, sm, Vp);
      const A tr = G::transport(Um, em);
      for (int k = 0; k < NG; ++k) G_.c[k] += (eh.c[k] - tr.c[k]) / ai;
    }
    acc[Q_G2] = norm2(G_);
    acc[Q_RHO2] = norm2(r);
    double gm = 0.0;
    for (int k = 0; k < NG; ++k) gm = fmax(gm, fabs(G_.c[k]));
    acc[Q_GMAX] = gm;
    acc[Q_BAD] = (bad || !isfinite(acc[Q_G2])) ? 1.0 : 0.0;
  }
  int z;
  uint32_t slot;
  col_map_block(m, blockIdx.x, z, slot);
  if (z >= g.nz) return;   // idle block (uniform over the block)
  const unsigned mask = (1u << Q_G2) | (1u << Q_RHO2) | (1u << Q_GMAX) | (1u << Q_UNIT) | (1u << Q_BAD);
  block_reduce_write<256>(acc, mask, partial + ((int64_t)z * nbx + slot) * NQ);
}

__global__ void __launch_bounds__(256) k_observe_finish(const double* __restrict__ partial, int nbx, Geom g,
                                                        StepConst c, double* __restrict__ out) {
  const int nz = g.nz;
  double loc[NQ];
  for (int q = 0; q < NQ; ++q) loc[q] = 0.0;
  const double inv_layer = 1.0 / (double)g.layer;
  for (int z = threadIdx.x; z < nz; z += blockDim.x) {
    double s[NQ];
    for (int q = 0; q < NQ; ++q) s[q] = 0.0;
    for (int b = 0; b < nbx; ++b)
      for (int q = 0; q < NQ; ++q) {
        double v = partial[((int64_t)z * nbx + b) * NQ + q];
        s[q] = (q == 6 || q == 7) ? fmax(s[q], v) : s[q] + v;
      }
    for (int q = 0; q < 4; ++q) out[q * nz + z] = s[q] * inv_layer;
    for (int q = 0; q < NQ; ++q) loc[q] = (q == 6 || q == 7) ? fmax(loc[q], s[q]) : loc[q] + s[q];
  }
  __shared__ double red[256][NQ];
  for (int q = 0; q < NQ; ++q) red[threadIdx.x][q] = loc[q];
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int q = 0; q < NQ; ++q)
        red[threadIdx.x][q] = (q == 6 || q == 7) ? fmax(red[threadIdx.x][q], red[threadIdx.x + w][q])
                                                 : red[threadIdx.x][q] + red[threadIdx.x + w][q];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double* o = out + 4 * nz;
    o[OBS_ENERGY] = c.a[0] * c.a[1] * c.a[2] * red[0][0];
    o[OBS_GAUSS_L2] = sqrt(red[0][4]);
    o[OBS_RHO_L2] = sqrt(red[0][5]);
    o[OBS_GAUSS_MAX] = red[0][6];
    o[OBS_UNITARITY] = red[0][7];
    o[OBS_NONFINITE] = red[0][8];
    o[OBS_GAUSS_REL] = red[0][5] > 0 ? sqrt(red[0][4] / red[0][5]) : sqrt(red[0][4]);
    o[7] = 0.0;
  }
}

template <typename G, typename T>
void launch_observe(const T* U, const T* E, const T* rhoA, const T* rhoB, const T* En, const Geom& g,
                    const StepConst& c, double* partial, double* out, hipStream_t st) {
  using Gd = typename GroupOf<G::NC, double>::type;
  const int nbx = obs_blocks_per_layer(g);
  // blocks start at multiples of 64 sites of a layer: rows lie in wavefronts when nt divides 64
  auto go = [&](auto kernel) {
    hipLaunchKernelGGL(kernel, dim3(nbx, g.nz), dim3(OBS_BS), 0, st, U, E, rhoA, rhoB, En, g, c, partial);
  };
  if (rows_in_wavefronts(g.nt)) En ? go(k_observe<Gd, T, true, true>) : go(k_observe<Gd, T, true, false>);
  else En ? go(k_observe<Gd, T, false, true>) : go(k_observe<Gd, T, false, false>);
  hipLaunchKernelGGL(k_observe_finish, dim3(1), dim3(256), 0, st, partial, nbx, g, c, out);
}

// ---- partial sums of the allocation-free observables call -------------------------
// A file-scope device array, one per GPU the library runs on (held until the process ends),
// for callers that cannot allocate; host code uses it only through the address that
// hipGetSymbolAddress returns for the current device, looked up once per device.
constexpr size_t OBS_STATIC_DOUBLES = (size_t)1 << 19;   // 4 MiB
static __device__ __align__(256) double g_obs_static[OBS_STATIC_DOUBLES];
constexpr int OBS_STATIC_MAX_DEVICES = 64;
static double* g_obs_static_ptr[OBS_STATIC_MAX_DEVICES];
static std::mutex g_obs_static_mu;

hipError_t observe_static_scratch(int device, double** ptr, size_t* capacity) {
  *capacity = OBS_STATIC_DOUBLES;
  if (device < 0 || device >= OBS_STATIC_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_obs_static_mu);
  if (!g_obs_static_ptr[device]) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(g_obs_static));
    if (cur != device) {
      const hipError_t e2 = hipSetDevice(cur);
      if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return e;
    g_obs_static_ptr[device] = (double*)p;
  }
  *ptr = g_obs_static_ptr[device];
  return hipSuccess;
}

// ---- pieces of the observing step (nt a multiple of 64: full column-map blocks) ----
bool fused_observe_geometry(const Geom& g) { return g.nt % 64 == 0; }
int fused_observe_blocks_per_layer(const Geom& g) { return col_map_slots_per_layer(col_map(g, 256)); }
template <typename G, typename T>
void launch_obs_gauss(const T* U, const T* E, const T* rhoA, const T* rhoB, const Geom& g, const StepConst& c,
                      double* partial, hipStream_t st) {
  using Gd = typename GroupOf<G::NC, double>::type;
  const ColMap m = col_map(g, 256);
  hipLaunchKernelGGL((k_obs_gauss<Gd, T>), dim3(col_map_blocks(g, m)), dim3(256), 0, st, U, E, rhoA, rhoB, g, c, m,
                     partial, fused_observe_blocks_per_layer(g));
}
void launch_observe_finish(const double* partial, int nbx, const Geom& g, const StepConst& c, double* out,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_observe_finish, dim3(1), dim3(256), 0, st, partial, nbx, g, c, out);
}

// ---- the observing step around a plain step (leapfrog; any geometry and precision) ----
// The observables of the state (U(t), E(t - dt/2), rho(t - dt/2)) that a step starts from,
// split around that step so that neither the step nor a separate pass forms the force twice:
//  - k_obs_pre, before the step, sums what that state fixes: the Gauss residual, |rho|^2,
//    B^2 from the forward plaquettes, the E(t - dt/2) halves of E^2 and of S_L, link
//    unitarity and the non-finite count.  It parks the two projections that S_L pairs with
//    E(t + dt/2), q_x = P(U_{x,z}) / (2 a_x a_z) and q_y = P(U_{y,z}) / (2 a_y a_z), in a
//    work buffer laid out as the x and y directions of an E field;
//  - the plain step writes E(t + dt/2), its hop current included;
//  - k_obs_post adds the E(t + dt/2) halves of E^2 and S_L to the same per-block sums.
// E^2 = (|E(t - dt/2)|^2 + |E(t + dt/2)|^2)/2 and S_L = sum_{i = x, y} Ebar_i . P(U_{i,z}) /
// (a_i a_z) are linear in the two half steps, so the sums split exactly (up to rounding).
// The plaquettes of an FP32 state are formed on links projected onto SU(N) in double
// precision, as in the standalone pass; unitarity and the Gauss residual read the links as
// stored.  Both passes cover a layer with obs_blocks_per_layer blocks, the same slots.
template <typename G, typename T, bool XS>
__global__ void __launch_bounds__(OBS_BS, 2) k_obs_pre(const T* __restrict__ U, const T* __restrict__ E,
                                                    const T* __restrict__ rhoA, const T* __restrict__ rhoB,
                                                    Geom g, StepConst c, T* __restrict__ Q,
                                                    double* __restrict__ partial) {
  using L = typename G::Link;   // double precision group
  using A = typename G::Alg;
  constexpr int NG = G::NG;
  const int64_t Vp = g.Vp;
  const int z = blockIdx.y;
  const int nbx = gridDim.x;
  constexpr bool PROJ = sizeof(T) == 4;
  constexpr int SLOT_BYTES = PROJ ? 3 * OwnProjLds<G>::NCH * OBS_BS * 16 : 3 * OwnSlot<G, T>::NCH * OBS_BS * 16;
  __shared__ double2 slot_mem[SLOT_BYTES / 16];
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
  // blocks start at multiples of 64 sites of the layer, so rows stay whole for XS
  const int64_t t = (int64_t)blockIdx.x * OBS_BS + threadIdx.x;
  if (t < g.layer) {
    const uint32_t s = (uint32_t)((int64_t)z * g.layer + t);
    Site x;
    x.x = (int)(t % g.nt);
    x.y = (int)(t / g.nt);
    x.z = z;
    const GlobalLinks<T> fetch{U, Vp};
    const ProjLinks<G, T> pfetch{fetch};
    // own links parked in LDS (projected onto SU(N) in double for FP32 storage), neighbour
    // links projected as they are read; a scheduling fence between the planes keeps the
    // compiler from hoisting every load to the top
    using OwnRaw = OwnLinks<G, T, OWN_LDS>;
    using Own = std::conditional_t<PROJ, OwnProjLds<G>, OwnRaw>;
    auto own = [&]() -> Own {
      if constexpr (PROJ) return Own(fetch, s, slot_mem, threadIdx.x);
      else return Own(fetch, s, (typename Vec16<T>::type*)slot_mem, threadIdx.x, OBS_BS);
    }();
    bool bad = false;
    XNbr xn;
    if constexpr (XS) xn = x_nbr(g, x);
    const uint32_t sx = idx(g, shifted(g, x, 0, +1));
    const uint32_t sy = idx(g, shifted(g, x, 1, +1));
    const uint32_t sz = idx(g, shifted(g, x, 2, +1));
    const double nc = (double)G::NC;
    const double inv_a2[3] = {1.0 / (c.a[0] * c.a[0]), 1.0 / (c.a[1] * c.a[1]), 1.0 / (c.a[2] * c.a[2])};
    double BL2, BT2 = 0.0, sl = 0.0, n2[3];
    {
      // (x, y): U_{x,y} = U_x(x) U_y(x+x) U_x(x+y)^dag U_y(x)^dag, its trace only
      L Oi, Oj, Nx, Nb;
      own(Oi, 0);
      own(Oj, 1);
      if constexpr (XS) Nx = pull_link(Oj, xn.ap);
      else pfetch(Nx, 1, sx);
      pfetch(Nb, 0, sy);
      double tr = 0.0;
      (void)G::proj_retr_mul_dag(G::mul_dag(G::mul(Oi, Nx), Nb), Oj, tr);
      BL2 = 4.0 * inv_a2[0] * inv_a2[1] * (nc - tr);
    }
    staple_fence<true>();
    // (x, z) and (y, z): traces for B_T^2, projections for S_L
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      L Oi, Oz, Nx, Nb;
      own(Oi, i);
      own(Oz, 2);
      if (i == 0) {
        if constexpr (XS) Nx = pull_link(Oz, xn.ap);
        else pfetch(Nx, 2, sx);
      } else {
        pfetch(Nx, 2, sy);
      }
      pfetch(Nb, i, sz);
      double tr = 0.0;
      const A p = G::proj_retr_mul_dag(G::mul_dag(G::mul(Oi, Nx), Nb), Oz, tr);
      BT2 += 4.0 * inv_a2[i] * inv_a2[2] * (nc - tr);
      const double h = 0.5 / (c.a[i] * c.a[2]);
      A q, eo;
      load_alg(eo, E, i, s, Vp);
#pragma unroll
      for (int k = 0; k < NG; ++k) {
        q.c[k] = h * p.c[k];
        sl += eo.c[k] * q.c[k];
        bad |= !isfinite(eo.c[k]);
      }
      n2[i] = norm2(eo);
      store_alg(q, Q, i, s, Vp);
      staple_fence<true>();
    }
    {
      A eo;
      load_alg(eo, E, 2, s, Vp);
#pragma unroll
      for (int k = 0; k < NG; ++k) bad |= !isfinite(eo.c[k]);
      n2[2] = norm2(eo);
    }
    const double EL2 = 0.5 * n2[2], ET2 = 0.5 * (n2[0] + n2[1]);
    acc[Q_EPS] = 0.5 * (EL2 + ET2 + BL2 + BT2);
    acc[Q_PL] = 0.5 * (ET2 + BT2 - EL2 - BL2);
    acc[Q_PT] = 0.5 * (EL2 + BL2);
    acc[Q_SL] = sl;
    // Gauss residual at (U(t), E(t - dt/2), rho(t - dt/2)); unitarity of the stored links
    A G_, r, rb;
    load_alg(r, rhoA, 0, site_index(g, x.x, x.y, slotA(z, c.offA, g.nz)), Vp);
    load_alg(rb, rhoB, 0, site_index(g, x.x, x.y, slotB(z, c.offB, g.nz)), Vp);
    for (int k = 0; k < NG; ++k) { r.c[k] += rb.c[k]; G_.c[k] = -r.c[k]; }
#pragma unroll 1
    for (int i = 0; i < 3; ++i) {
      const double ai = i == 0 ? c.a[0] : (i == 1 ? c.a[1] : c.a[2]);
      const uint32_t sm = idx(g, shifted(g, x, i, -1));
      L Um;
      load_link(Um, U, i, sm, Vp);
      // every link is read here once, as U_i(x - i) of x = y + i: the unitarity maximum
      const double uv = G::unit_violation(Um);
      bad |= !isfinite(uv);
      acc[Q_UNIT] = fmax(acc[Q_UNIT], uv);
      A eh, em;
      load_alg(eh, E, i, s, Vp);
      load_alg(em, E, i, sm, Vp);
      const A tt = G::transport(Um, em);
      for (int k = 0; k < NG; ++k) G_.c[k] += (eh.c[k] - tt.c[k]) / ai;
    }
    acc[Q_G2] = norm2(G_);
    acc[Q_RHO2] = norm2(r);
    double gm = 0.0;
    for (int k = 0; k < NG; ++k) gm = fmax(gm, fabs(G_.c[k]));
    acc[Q_GMAX] = gm;
    bad |= !isfinite(acc[Q_EPS]) || !isfinite(acc[Q_G2]);
    acc[Q_BAD] = bad ? 1.0 : 0.0;
  }
  block_reduce_write<OBS_BS>(acc, Q_ALL, partial + ((int64_t)z * nbx + blockIdx.x) * NQ);
}

template <typename G, typename T>
__global__ void __launch_bounds__(OBS_BS) k_obs_post(const T* __restrict__ E, const T* __restrict__ Q, Geom g,
                                                     double* __restrict__ partial) {
  using A = typename G::Alg;
  constexpr int NG = G::NG;
  const int64_t Vp = g.Vp;
  const int z = blockIdx.y;
  const int nbx = gridDim.x;
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
  const int64_t t = (int64_t)blockIdx.x * OBS_BS + threadIdx.x;
  if (t < g.layer) {
    const uint32_t s = (uint32_t)((int64_t)z * g.layer + t);
    double n2[3], sl = 0.0;
    bool bad = false;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      A en;
      load_alg_own(en, E, i, s, Vp);
#pragma unroll
      for (int k = 0; k < NG; ++k) bad |= !isfinite(en.c[k]);
      n2[i] = norm2(en);
      if (i < 2) {
        A q;
        load_alg_own(q, Q, i, s, Vp);
#pragma unroll
        for (int k = 0; k < NG; ++k) sl += en.c[k] * q.c[k];
      }
    }
    const double EL2 = 0.5 * n2[2], ET2 = 0.5 * (n2[0] + n2[1]);
    acc[Q_EPS] = 0.5 * (EL2 + ET2);
    acc[Q_PL] = 0.5 * (ET2 - EL2);
    acc[Q_PT] = 0.5 * EL2;
    acc[Q_SL] = sl;
    acc[Q_BAD] = (bad || !isfinite(sl)) ? 1.0 : 0.0;
  }
  constexpr unsigned M = (1u << Q_EPS) | (1u << Q_PL) | (1u << Q_PT) | (1u << Q_SL) | (1u << Q_BAD);
  block_reduce_write<OBS_BS, M>(acc, M, partial + ((int64_t)z * nbx + blockIdx.x) * NQ);
}

size_t obs_split_scratch_elems(const Geom& g, int ng) { return (size_t)2 * ng * g.Vp; }

template <typename G, typename T>
void launch_obs_pre(const T* U, const T* E, const T* rhoA, const T* rhoB, const Geom& g, const StepConst& c, T* Q,
                    double* partial, hipStream_t st) {
  using Gd = typename GroupOf<G::NC, double>::type;
  const dim3 grid(obs_blocks_per_layer(g), g.nz);
  if (rows_in_wavefronts(g.nt))
    hipLaunchKernelGGL((k_obs_pre<Gd, T, true>), grid, dim3(OBS_BS), 0, st, U, E, rhoA, rhoB, g, c, Q, partial);
  else
    hipLaunchKernelGGL((k_obs_pre<Gd, T, false>), grid, dim3(OBS_BS), 0, st, U, E, rhoA, rhoB, g, c, Q, partial);
}
template <typename G, typename T>
void launch_obs_post(const T* E, const T* Q, const Geom& g, const StepConst& c, double* partial, double* out,
                     hipStream_t st) {
  using Gd = typename GroupOf<G::NC, double>::type;
  const int nbx = obs_blocks_per_layer(g);
  hipLaunchKernelGGL((k_obs_post<Gd, T>), dim3(nbx, g.nz), dim3(OBS_BS), 0, st, E, Q, g, partial);
  hipLaunchKernelGGL(k_observe_finish, dim3(1), dim3(256), 0, st, partial, nbx, g, c, out);
}

// ---- local rest frame per layer (Sec. 4) ----------------------------------------
// eps_loc and the frame velocity v along +z from the timelike eigenvector of the (t, z)
// block of T^mu_nu, [[eps, -S_L], [S_L, -p_L]]:  S_L v^2 - (eps + p_L) v + S_L = 0.
__global__ void k_rest_frame(const double* __restrict__ obs, int nz, double* __restrict__ out) {
  const int z = blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= nz) return;
  const double eps = obs[z], pL = obs[nz + z], SL = obs[3 * nz + z];
  const double s = eps + pL;
  const double root = sqrt(fmax(s * s - 4.0 * SL * SL, 0.0));
  const double den = s + root;
  const double v = den > 0.0 ? 2.0 * SL / den : 0.0;
  out[z] = eps - SL * v;
  out[nz + z] = v;
}
void launch_rest_frame(const double* obs, int nz, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_rest_frame, dim3((unsigned)((nz + 255) / 256)), dim3(256), 0, st, obs, nz, out);
}

// ---- event averages of the slices over a batch (Sec. 2 eq. ev; Sec. 4) ----------------
// obs: the events' observables buffers, event e at obs + ev[e].off (4 nz_e slices first).
// Output element t < cls_total: class averages (class k's [4][nz_k] block at cls_off[k]);
// after that the common grid [4][n_grid] of relative position z / nz, bin b = floor(z n_grid / nz).
__global__ void k_batch_average(const double* __restrict__ obs, const BatchObsEvent* __restrict__ ev, int n_events,
                                const int* __restrict__ cls_nz, const int* __restrict__ cls_off,
                                const int* __restrict__ cls_count, int n_cls, int cls_total, int n_grid,
                                double* __restrict__ cls_out, double* __restrict__ grid_out) {
  const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (t < cls_total) {
    int k = 0;
    while (k + 1 < n_cls && t >= cls_off[k + 1]) ++k;
    const int nz = cls_nz[k], r = t - cls_off[k], q = r / nz, z = r % nz;
    double sum = 0.0;
    for (int e = 0; e < n_events; ++e)
      if (ev[e].cls == k) sum += obs[ev[e].off + (int64_t)q * nz + z];
    cls_out[t] = sum / (double)cls_count[k];
  } else if (t < cls_total + 4 * n_grid) {
    const int r = t - cls_total, q = r / n_grid, b = r % n_grid;
    double sum = 0.0;
    for (int e = 0; e < n_events; ++e) {
      const int nz = ev[e].nz;
      // layers z with floor(z n_grid / nz) = b: z in [ceil(b nz / n_grid), ceil((b + 1) nz / n_grid))
      const int z0 = (int)(((int64_t)b * nz + n_grid - 1) / n_grid);
      const int z1 = (int)(((int64_t)(b + 1) * nz + n_grid - 1) / n_grid);
      double m = 0.0;
      for (int z = z0; z < z1; ++z) m += obs[ev[e].off + (int64_t)q * nz + z];
      sum += m / (double)(z1 - z0);
    }
    grid_out[r] = sum / (double)n_events;
  }
}
void launch_batch_average(const double* obs, const BatchObsEvent* ev, int n_events, const int* cls_nz,
                          const int* cls_off, const int* cls_count, int n_cls, int cls_total, int n_grid,
                          double* cls_out, double* grid_out, hipStream_t st) {
  const int n = cls_total + 4 * n_grid;
  hipLaunchKernelGGL(k_batch_average, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, obs, ev, n_events, cls_nz,
                     cls_off, cls_count, n_cls, cls_total, n_grid, cls_out, grid_out);
}

// ---- current of the next step (tests) --------------------------------------
template <typename G, typename T>
__global__ void k_current(const T* __restrict__ U, const T* __restrict__ rhoA, const T* __restrict__ rhoB,
                          Geom g, StepConst c, T* __restrict__ j) {
  using L = typename G::Link;
  using A = typename G::Alg;
  constexpr int NG = G::NG;
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  const int64_t Vp = g.Vp;
  const int x = (int)(s % g.nt), y = (int)((s / g.nt) % g.nt), z = (int)(s / g.layer);
  A jz = G::alg_zero();
  if (c.hop) {
    L Uz;
    load_link(Uz, U, 2, s, Vp);
    A rb, ra;
    load_alg(rb, rhoB, 0, site_index(g, x, y, slotB(z, c.offB, g.nz)), Vp);
    load_alg(ra, rhoA, 0, site_index(g, x, y, slotA(wrap_add(z, 1, g.nz), c.offA, g.nz)), Vp);
    A ran = G::transport_inv(Uz, ra);
    const typename G::Real k = (typename G::Real)(c.a[2] / c.dt);
    for (int q = 0; q < NG; ++q) jz.c[q] = k * (ran.c[q] - rb.c[q]);
  }
  // plain structure-of-arrays output j[(i * NG + a) * V + s]
  const int64_t V = g.V;
#pragma unroll
  for (int q = 0; q < NG; ++q) {
    j[(int64_t)q * V + s] = T(0);
    j[(int64_t)(NG + q) * V + s] = T(0);
    j[(int64_t)(2 * NG + q) * V + s] = (T)jz.c[q];
  }
}

template <typename G, typename T>
void launch_current(const T* U, const T* rhoA, const T* rhoB, const Geom& g, const StepConst& c, T* j,
                    hipStream_t st) {
  const int bs = 256;
  hipLaunchKernelGGL((k_current<G, T>), dim3((unsigned)((g.V + bs - 1) / bs)), dim3(bs), 0, st, U, rhoA, rhoB, g, c, j);
}

// ---- FP64 reunitarisation ----------------------------------------------------
template <typename Gd, typename T>
__global__ void k_reunit(T* __restrict__ U, Geom g) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  const int64_t Vp = g.Vp;
  for (int i = 0; i < 3; ++i) {
    typename Gd::Link l;
    load_link(l, U, i, s, Vp);
    store_link(Gd::reunit(l), U, i, s, Vp);
  }
}

template <typename G, typename T>
void launch_reunit(T* U, const Geom& g, hipStream_t st) {
  using Gd = typename GroupOf<G::NC, double>::type;
  const int bs = 256;
  hipLaunchKernelGGL((k_reunit<Gd, T>), dim3((unsigned)((g.V + bs - 1) / bs)), dim3(bs), 0, st, U, g);
}

#define GL_INST(G, T)                                                                                       \
  template void launch_observe<G, T>(const T*, const T*, const T*, const T*, const T*, const Geom&,             \
                                     const StepConst&,                                                      \
                                     double*, double*, hipStream_t);                                        \
  template void launch_current<G, T>(const T*, const T*, const T*, const Geom&, const StepConst&, T*,      \
                                     hipStream_t);                                                          \
  template void launch_reunit<G, T>(T*, const Geom&, hipStream_t);                                        \
  template void launch_obs_gauss<G, T>(const T*, const T*, const T*, const T*, const Geom&, const StepConst&, \
                                       double*, hipStream_t);                                             \
  template void launch_obs_pre<G, T>(const T*, const T*, const T*, const T*, const Geom&, const StepConst&, T*, \
                                     double*, hipStream_t);                                               \
  template void launch_obs_post<G, T>(const T*, const T*, const Geom&, const StepConst&, double*, double*,   \
                                      hipStream_t);
GL_INST(Su2<double>, double)
GL_INST(Su3<double>, double)
GL_INST(Su2<float>, float)
GL_INST(Su3<float>, float)

}  // namespace gl
