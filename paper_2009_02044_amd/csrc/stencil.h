// Plaquette sums of the Wilson-action force (Sec. 3, eqs. lattice_1 and plaquette).
#pragma once
#include "lattice.h"

namespace gl {

// Scheduling fence between plaquette groups: limits how many links the compiler keeps in
// flight at once.  Off for the plain step (no gain there); on where ON is set, for the
// observing step, whose extra state keeps it at the edge of its register budget (with the
// link unitarity measured in the Gauss pass instead, it runs as fast without the fence).
#ifndef GL_STAPLE_FENCE
#define GL_STAPLE_FENCE 0
#endif
template <bool ON = false> __device__ __forceinline__ void staple_fence() {
  if constexpr (ON || GL_STAPLE_FENCE) __builtin_amdgcn_sched_barrier(0);
}

// Link source for the plaquette sums: fetch(l, d, s) sets l = U_d at site s.
template <typename T> struct GlobalLinks {
  const T* __restrict__ U;
  int64_t Vp;
  template <typename L> __device__ __forceinline__ void operator()(L& l, int d, uint32_t s) const {
    load_link(l, U, d, s, Vp);
  }
};

template <typename R> __device__ __forceinline__ void select3(M3<R>& l, int d, const M3<R>& a, const M3<R>& b,
                                                             const M3<R>& c) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      l.re[i][j] = d == 0 ? a.re[i][j] : (d == 1 ? b.re[i][j] : c.re[i][j]);
      l.im[i][j] = d == 0 ? a.im[i][j] : (d == 1 ? b.im[i][j] : c.im[i][j]);
    }
}
template <typename R> __device__ __forceinline__ void select3(Q2<R>& l, int d, const Q2<R>& a, const Q2<R>& b,
                                                             const Q2<R>& c) {
#pragma unroll
  for (int k = 0; k < 4; ++k) l.q[k] = d == 0 ? a.q[k] : (d == 1 ? b.q[k] : c.q[k]);
}
// Where the site's own three links come from each time a plaquette or the link update
// needs them: loaded again from memory (OWN_REFETCH), kept in registers (OWN_REGS), or
// parked once in a per-thread LDS slot and rebuilt from there (OWN_LDS; a thread reads
// only its own slot, so no barrier is needed).  LDS slot layout: chunk q of direction d
// of thread t at [(d NCH + q) TB + t], a wavefront's access covering 64 consecutive
// 16-byte words.
enum { OWN_REFETCH = 0, OWN_REGS = 1, OWN_LDS = 2 };
template <typename G, typename T> struct OwnSlot {
  using V16 = typename Vec16<T>::type;
  static constexpr int W = StoredWidth<typename G::Link>::value;
  static constexpr int NCH = W * (int)sizeof(T) / 16;   // 16-byte chunks per stored link
  static_assert(NCH * 16 == W * (int)sizeof(T), "stored link is not a whole number of chunks");
};
template <typename G, typename T, int MODE> struct OwnLinks;
template <typename G, typename T> struct OwnLinks<G, T, OWN_REGS> {
  typename G::Link O[3];
  __device__ __forceinline__ OwnLinks(const GlobalLinks<T>& f, uint32_t s, typename Vec16<T>::type*, uint32_t,
                                      uint32_t) {
#pragma unroll
    for (int d = 0; d < 3; ++d) f(O[d], d, s);
  }
  // d may be a run-time value: select member by member (no indexed register array)
  __device__ __forceinline__ void operator()(typename G::Link& l, int d) const { select3(l, d, O[0], O[1], O[2]); }
};
template <typename G, typename T> struct OwnLinks<G, T, OWN_REFETCH> {
  GlobalLinks<T> f;
  uint32_t s;
  __device__ __forceinline__ OwnLinks(const GlobalLinks<T>& f_, uint32_t s_, typename Vec16<T>::type*, uint32_t,
                                      uint32_t)
      : f(f_), s(s_) {}
  // the site index passes through an empty asm statement so that the compiler sees each
  // re-fetch as a new load and does not merge them into one long-lived copy
  __device__ __forceinline__ void operator()(typename G::Link& l, int d) const {
    uint32_t t = s;
    asm volatile("" : "+v"(t));
    f(l, d, t);
  }
};
template <typename G, typename T> struct OwnLinks<G, T, OWN_LDS> {
  using Sl = OwnSlot<G, T>;
  using V16 = typename Sl::V16;
  V16* lds;
  uint32_t t, TB;
  __device__ __forceinline__ OwnLinks(const GlobalLinks<T>& f, uint32_t s, V16* lds_, uint32_t t_, uint32_t TB_)
      : lds(lds_), t(t_), TB(TB_) {
    const uint32_t l = s % RB;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const char* rec = (const char*)field_dir(f.U, d, Sl::W, f.Vp) + (uint64_t)(s / RB) * RecShape<T, Sl::W>::BYTES;
#pragma unroll
      for (int q = 0; q < Sl::NCH; ++q) lds[(d * Sl::NCH + q) * TB + t] = *(const V16*)(rec + q * (RB * 16) + l * 16);
    }
  }
  // (the slot index is laundered like the site index of OWN_REFETCH)
  __device__ __forceinline__ void operator()(typename G::Link& l, int d) const {
    constexpr int VW = Rec<T>::VW;
    uint32_t tt = t;
    asm volatile("" : "+v"(tt));
    typename G::Real v[Sl::W];
#pragma unroll
    for (int q = 0; q < Sl::NCH; ++q) {
      const V16 x = lds[(d * Sl::NCH + q) * TB + tt];
      const T* e = (const T*)&x;
#pragma unroll
      for (int k = 0; k < VW; ++k) v[q * VW + k] = (typename G::Real)e[k];
    }
    link_from_stored(l, v);
  }
};

// ---- x neighbours from other lanes --------------------------------------------
// When nt divides 64 and a wavefront holds 64 consecutive sites starting at a multiple
// of 64, every x row lies inside one wavefront: the link at x +- e_x of a site is held
// by the lane 1 apart, or nt - 1 apart across the periodic end of the row.  It is
// pulled through the LDS crossbar (ds_bpermute, no LDS allocation).
struct XNbr {
  int ap, am;   // byte address (4 x source lane) of the lane holding x + e_x / x - e_x
};
__device__ __forceinline__ XNbr x_nbr(const Geom& g, Site x) {
  const int lane = (int)(threadIdx.x & 63u);
  XNbr n;
  n.ap = 4 * (lane + (x.x + 1 < g.nt ? 1 : 1 - g.nt));
  n.am = 4 * (lane + (x.x > 0 ? -1 : g.nt - 1));
  return n;
}
GL_HD bool rows_in_wavefronts(int nt) { return nt > 0 && nt <= 64 && (64 % nt) == 0; }
__device__ __forceinline__ float lane_pull(float v, int a) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(a, __float_as_int(v)));
}
__device__ __forceinline__ double lane_pull(double v, int a) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_bpermute(a, (int)b);
  const int hi = __builtin_amdgcn_ds_bpermute(a, (int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <typename R> __device__ __forceinline__ M3<R> pull_link(const M3<R>& v, int a) {
  M3<R> r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) { r.re[i][j] = lane_pull(v.re[i][j], a); r.im[i][j] = lane_pull(v.im[i][j], a); }
  return r;
}
template <typename R> __device__ __forceinline__ Q2<R> pull_link(const Q2<R>& v, int a) {
  Q2<R> r;
#pragma unroll
  for (int k = 0; k < 4; ++k) r.q[k] = lane_pull(v.q[k], a);
  return r;
}

template <typename A> __device__ __forceinline__ A pull_alg(const A& v, int a) {
  constexpr int NG = sizeof(v.c) / sizeof(v.c[0]);
  A r;
#pragma unroll
  for (int k = 0; k < NG; ++k) r.c[k] = lane_pull(v.c[k], a);
  return r;
}

// ---- force from plaquettes --------------------------------------------------------
// f_i = sum_{j != i} w_j [ P(U_{i,j}(x)) + P(U_{i,-j}(x)) ],  w_j = a_j^-2, so that
// F_i = -f_i / a_i.  Plaquette by plaquette: a forward plaquette serves two
// directions, U_{j,i}(x) = U_{i,j}(x)^dag and P(M^dag) = -P(M); the backward
// plaquettes that share a link are taken together.  With XS (rows in wavefronts) the
// links at x +- e_x come from the neighbouring lanes, so a site loads 15 links, and the
// backward plaquettes in the -x direction are the neighbour lane's forward ones carried
// over by one link: U_{i,-x}(x) = W^dag U_{x,i}(x - e_x) W, W = U_x(x - e_x), and
// P(W^dag M W) = W^dag P(M) W.
// The forward plaquettes at x, for the observables: a hook object receives, for plane K
// (0 = (x, y), 1 = (x, z), 2 = (y, z)), the projection and real trace of U_{x,y}, U_{x,z}
// or U_{y,z}, with the force term that is complete at that point (f_x for K = 1, f_y
// for K = 2; see the group order below).  PlaqObs keeps them for later use.
template <typename G> struct PlaqObs {
  typename G::Alg p[3];
  typename G::Real tr[3];
  template <int K>
  __device__ __forceinline__ void plane(const typename G::Alg& pk, typename G::Real t, const typename G::Alg&) {
    p[K] = pk;
    tr[K] = t;
  }
};

// own(l, d) sets l = U_d(x) (kept in registers or fetched again).  With OBS the forward
// plaquettes are also handed to po.
template <typename G, bool XS, bool OBS = false, typename F, typename OwnF, typename Obs = PlaqObs<G>>
__device__ __forceinline__ void plaquette_forces(const F& fetch, const OwnF& own, const Geom& g, Site x,
                                                 const double* inv_a2, typename G::Alg (&f)[3],
                                                 Obs* po = nullptr) {
  using L = typename G::Link;
  using Ag = typename G::Alg;
  using R = typename G::Real;
  constexpr int NG = G::NG;
  const R w0 = (R)inv_a2[0], w1 = (R)inv_a2[1], w2 = (R)inv_a2[2];
  XNbr xn;
  if (XS) xn = x_nbr(g, x);
  // link U_d(y +- e_x) where every lane holds v = U_d(y) for its own y
  auto xs = [&](const L& v, Site y, int d, int dir) -> L {
    if constexpr (XS) {
      return pull_link(v, dir > 0 ? xn.ap : xn.am);
    } else {
      L r;
      fetch(r, d, idx(g, shifted(g, y, 0, dir)));
      return r;
    }
  };
  auto acc = [&](Ag& a, const Ag& p, R w) {
#pragma unroll
    for (int k = 0; k < NG; ++k) a.c[k] = fmx(w, p.c[k], a.c[k]);
  };
#pragma unroll
  for (int i = 0; i < 3; ++i) f[i] = G::alg_zero();
  const Site xpy = shifted(g, x, 1, +1), xpz = shifted(g, x, 2, +1);
  const Site xmy = shifted(g, x, 1, -1), xmz = shifted(g, x, 2, -1);
  auto b_xy = [&]() {
    // plane (x, y): forward, and backward for y in -x
    L O0, O1, A, B;
    own(O0, 0);
    own(O1, 1);
    fetch(B, 0, idx(g, xpy));                                 // U_0(x+y)
    A = xs(O1, x, 1, +1);                                     // U_1(x+x)
    const L M2 = G::mul_dag(G::mul(O0, A), B);
    R tr = R(0);
    const Ag p = OBS ? G::proj_retr_mul_dag(M2, O1, tr) : G::proj_mul_dag(M2, O1);
    acc(f[0], p, w1);
    acc(f[1], p, -w0);
    if constexpr (OBS) po->template plane<0>(p, tr, f[0]);
    staple_fence<OBS>();
    if constexpr (XS) {
      // U_{1,-0}(x) = W^dag U_{0,1}(x-x) W with W = U_0(x-x): transport the neighbour
      // lane's forward plaquette instead of forming the backward one
      acc(f[1], G::transport(pull_link(O0, xn.am), pull_alg(p, xn.am)), w0);
    } else {
      const L A2 = xs(B, xpy, 0, -1);                         // U_0(x+y-x)
      const L B2 = xs(O1, x, 1, -1);                          // U_1(x-x)
      const L C2 = xs(O0, x, 0, -1);                          // U_0(x-x)
      acc(f[1], G::proj_mul(G::mul_dag(O1, G::mul(B2, A2)), C2), w0);
    }
    staple_fence<OBS>();
  };
  auto b_xz = [&]() {
    // plane (x, z): forward, and backward for z in -x
    L O0, O2, A, B;
    own(O0, 0);
    own(O2, 2);
    fetch(B, 0, idx(g, xpz));                                 // U_0(x+z)
    A = xs(O2, x, 2, +1);                                     // U_2(x+x)
    const L M2 = G::mul_dag(G::mul(O0, A), B);
    R tr = R(0);
    const Ag p = OBS ? G::proj_retr_mul_dag(M2, O2, tr) : G::proj_mul_dag(M2, O2);
    acc(f[0], p, w2);
    acc(f[2], p, -w0);
    if constexpr (OBS) po->template plane<1>(p, tr, f[0]);   // f_x complete
    staple_fence<OBS>();
    if constexpr (XS) {
      acc(f[2], G::transport(pull_link(O0, xn.am), pull_alg(p, xn.am)), w0);
    } else {
      const L A2 = xs(B, xpz, 0, -1);                         // U_0(x+z-x)
      const L B2 = xs(O2, x, 2, -1);                          // U_2(x-x)
      const L C2 = xs(O0, x, 0, -1);                          // U_0(x-x)
      acc(f[2], G::proj_mul(G::mul_dag(O2, G::mul(B2, A2)), C2), w0);
    }
    staple_fence<OBS>();
  };
  auto b_yz = [&]() {
    // plane (y, z): forward
    L O1, O2, A, B;
    own(O1, 1);
    own(O2, 2);
    fetch(A, 2, idx(g, xpy));                                 // U_2(x+y)
    fetch(B, 1, idx(g, xpz));                                 // U_1(x+z)
    const L M2 = G::mul_dag(G::mul(O1, A), B);
    R tr = R(0);
    const Ag p = OBS ? G::proj_retr_mul_dag(M2, O2, tr) : G::proj_mul_dag(M2, O2);
    acc(f[1], p, w2);
    acc(f[2], p, -w1);
    if constexpr (OBS) po->template plane<2>(p, tr, f[1]);   // f_y complete
    staple_fence<OBS>();
  };
  auto b_my = [&]() {
    // backward in -y for x and z, sharing U_1(x-y)
    L Y1, O, A, B;
    fetch(Y1, 1, idx(g, xmy));                                // U_1(x-y)
    fetch(B, 0, idx(g, xmy));                                 // U_0(x-y)
    own(O, 0);
    A = xs(Y1, xmy, 1, +1);                                   // U_1(x+x-y)
    acc(f[0], G::proj_mul(G::mul_dag(O, G::mul(B, A)), Y1), w1);
    staple_fence<OBS>();
    own(O, 2);
    fetch(A, 1, idx(g, shifted(g, xpz, 1, -1)));              // U_1(x+z-y)
    fetch(B, 2, idx(g, xmy));                                 // U_2(x-y)
    acc(f[2], G::proj_mul(G::mul_dag(O, G::mul(B, A)), Y1), w1);
    staple_fence<OBS>();
  };
  auto b_mz = [&]() {
    // backward in -z for x and y, sharing U_2(x-z)
    L Z2, O, A, B;
    fetch(Z2, 2, idx(g, xmz));                                // U_2(x-z)
    fetch(B, 0, idx(g, xmz));                                 // U_0(x-z)
    own(O, 0);
    A = xs(Z2, xmz, 2, +1);                                   // U_2(x+x-z)
    acc(f[0], G::proj_mul(G::mul_dag(O, G::mul(B, A)), Z2), w2);
    staple_fence<OBS>();
    own(O, 1);
    fetch(A, 2, idx(g, shifted(g, xpy, 2, -1)));              // U_2(x+y-z)
    fetch(B, 1, idx(g, xmz));                                 // U_1(x-z)
    acc(f[1], G::proj_mul(G::mul_dag(O, G::mul(B, A)), Z2), w2);
    staple_fence<OBS>();
  };
  // Order of the plaquette groups (the force sums in this order).  The -z group first:
  // its links of layer z - 1 are then loaded while the work-groups of that layer load
  // them as their own, so they are still in the L2.  The -y group before the forward
  // (x, z) and (y, z) groups: f_x is then complete once the (x, z) plaquette is formed and
  // f_y once the (y, z) one is, so an observer consumes each projection at once.
  b_mz();
  b_xy();
  b_my();
  b_xz();
  b_yz();
}

}  // namespace gl
