// Semi-implicit scheme: the slice force f1(A, B) of every link in one pass (Sec. 3, fig. wilson;
// the potential between two time slices and the derivative rule are stated in semi.hip).
//
// A wavefront owns a column of 64 consecutive sites of a layer (nt divides 64 and
// nt >= 8: whole x rows, x neighbours in adjacent lanes) and marches along z through
// a chunk of layers.  At each layer it forms the plaquette-like loops based at its sites
// once and hands each loop's derivative to the links that carry it:
//   * links of its own site: accumulated directly;
//   * links at x + e_x (factor 1 of an (x, y) or (x, z) loop): pulled by the next lane;
//   * links at x + e_z (factor 2 of an (x, z) or (y, z) loop): carried to the next layer;
//   * links at x + e_y (factor 2 of an (x, y) loop, factor 1 of a (y, z) loop): the site
//     above forms those loops again at its base - e_y (another wavefront's column).
// Per site and slice 11 distinct links are read (against about 75 when every link forms
// all its loops), and about 85 matrix products are formed (against about 135).  With
// MODE = 1 the pass also completes the fixed-point iteration of each link as soon as its
// force is complete (E' = Ebase + dt f1, under-relaxed, new trial link), so the force is
// never stored; MODE = 0 stores f1 (the per-step term f1(U(t), U(t - dt))).
#include "internal.h"
#include "stencil.h"

namespace gl {

namespace {

// components of M + M^dag (hermitian; its traceless part)
template <typename G> __device__ __forceinline__ typename G::Alg hsum(const typename G::Link& m) {
  typename G::Link h = m;
  G::add_to(h, G::dag(m), (typename G::Real)(G::NC == 3 ? 1 : -1));
  return G::alg_from_herm(h);
}
template <typename G> __device__ __forceinline__ typename G::Link yP(const typename G::Link& c) {
  return G::herm_from_alg(G::proj(c));
}
// loop F0 F1 F2^dag F3^dag
template <typename G>
__device__ __forceinline__ typename G::Link loop4(const typename G::Link& f0, const typename G::Link& f1,
                                                  const typename G::Link& f2, const typename G::Link& f3) {
  return G::mul_dag(G::mul_dag(G::mul(f0, f1), f2), f3);
}
template <typename A, typename R> __device__ __forceinline__ void axpy(A& acc, R s, const A& x) {
  constexpr int NG = sizeof(acc.c) / sizeof(acc.c[0]);
#pragma unroll
  for (int k = 0; k < NG; ++k) acc.c[k] = fmx(s, x.c[k], acc.c[k]);
}
// Components of H = M + M^dag for M = C Y (LEFT = false) or M = Y C (LEFT = true), with Y the
// hermitian matrix of the algebra element y, without forming M: only the 15 entries of M
// that H's traceless part reads, and Y's real diagonal taken as real (a general product
// would multiply its zero imaginary parts too).  SU(3); SU(2) takes the general route.
template <bool LEFT, typename R>
__device__ __forceinline__ Alg3<R> hs_herm(const M3<R>& C, const Alg3<R>& y) {
  const typename Su3<R>::Herm q = Su3<R>::herm_c(y, R(1));
  // Y_kj = (yr, yi)
  auto Y = [&](int k, int j, R& yr, R& yi) {
    if (k == j) { yr = q.d[j]; yi = R(0); return; }
    const int n = (k == 0 || j == 0) ? ((k == 1 || j == 1) ? 0 : 1) : 2;
    yr = q.r[n];
    yi = k < j ? q.i[n] : -q.i[n];
  };
  // entry (p, j) of M, real (want_im false) or imaginary part
  auto ent = [&](int p, int j, bool want_im) -> R {
    R acc = R(0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      R yr, yi;
      R cr, ci;
      if (LEFT) {   // M_pj = sum_k Y_pk C_kj
        Y(p, k, yr, yi);
        cr = C.re[k][j];
        ci = C.im[k][j];
        const bool real_y = p == k;
        if (!want_im) {
          acc = fmx(yr, cr, acc);
          if (!real_y) acc = fmx(-yi, ci, acc);
        } else {
          acc = fmx(yr, ci, acc);
          if (!real_y) acc = fmx(yi, cr, acc);
        }
      } else {      // M_pj = sum_k C_pk Y_kj
        Y(k, j, yr, yi);
        cr = C.re[p][k];
        ci = C.im[p][k];
        const bool real_y = k == j;
        if (!want_im) {
          acc = fmx(cr, yr, acc);
          if (!real_y) acc = fmx(-ci, yi, acc);
        } else {
          acc = fmx(ci, yr, acc);
          if (!real_y) acc = fmx(cr, yi, acc);
        }
      }
    }
    return acc;
  };
  const R is3 = R(0.57735026918962576451);
  const R m00 = ent(0, 0, false), m11 = ent(1, 1, false), m22 = ent(2, 2, false);
  Alg3<R> r;
  r.c[0] = R(2) * (ent(0, 1, false) + ent(1, 0, false));
  r.c[1] = R(2) * (ent(1, 0, true) - ent(0, 1, true));
  r.c[2] = R(2) * (m00 - m11);
  r.c[3] = R(2) * (ent(0, 2, false) + ent(2, 0, false));
  r.c[4] = R(2) * (ent(2, 0, true) - ent(0, 2, true));
  r.c[5] = R(2) * (ent(1, 2, false) + ent(2, 1, false));
  r.c[6] = R(2) * (ent(2, 1, true) - ent(1, 2, true));
  r.c[7] = R(2) * (m00 + m11 - R(2) * m22) * is3;
  return r;
}
template <bool LEFT, typename R>
__device__ __forceinline__ Alg2<R> hs_herm(const Q2<R>& C, const Alg2<R>& y) {
  using G = Su2<R>;
  const Q2<R> Y = G::herm_from_alg(y);
  return hsum<G>(LEFT ? G::mul(Y, C) : G::mul(C, Y));
}

// Full matrices in 18-wide records (the loop cache): component 2 (3 r + k) + {re, im}; SU(2)
// loops are quaternions (4 wide).
template <typename L> struct FullWidth;
template <typename R> struct FullWidth<M3<R>> { static constexpr int value = 18; };
template <typename R> struct FullWidth<Q2<R>> { static constexpr int value = 4; };
template <typename R, typename T>
__device__ __forceinline__ void store_full(const M3<R>& m, T* f, int plane, uint32_t s, int64_t Vp) {
  R v[18];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) { v[2 * (3 * r + k)] = m.re[r][k]; v[2 * (3 * r + k) + 1] = m.im[r][k]; }
  store_comps<R, T, 18>(v, field_dir(f, plane, 18, Vp), s);
}
template <typename R, typename T>
__device__ __forceinline__ void store_full(const Q2<R>& m, T* f, int plane, uint32_t s, int64_t Vp) {
  store_comps<R, T, 4>(m.q, field_dir(f, plane, 4, Vp), s);
}
template <typename R, typename T>
__device__ __forceinline__ void load_full(M3<R>& m, const T* f, int plane, uint32_t s, int64_t Vp) {
  R v[18];
  load_comps<R, T, 18>(v, field_dir(f, plane, 18, Vp), s);
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) { m.re[r][k] = v[2 * (3 * r + k)]; m.im[r][k] = v[2 * (3 * r + k) + 1]; }
}
template <typename R, typename T>
__device__ __forceinline__ void load_full(Q2<R>& m, const T* f, int plane, uint32_t s, int64_t Vp) {
  load_comps<R, T, 4>(m.q, field_dir(f, plane, 4, Vp), s);
}
// Accumulator of an algebra element that lives in registers (LDS = false) or in a
// per-thread slot of the work-group's LDS (LDS = true; a thread only touches its own slot,
// so no barrier is needed): components k at p[k * MARCH_BS].
template <typename Ag, typename R, bool LDS> struct Acc;
template <typename Ag, typename R> struct Acc<Ag, R, false> {
  Ag v;
  __device__ __forceinline__ Ag get() const { return v; }
  __device__ __forceinline__ void set(const Ag& x) { v = x; }
  __device__ __forceinline__ void add(R s, const Ag& x) { axpy(v, s, x); }
  __device__ __forceinline__ void scale(R s) {
    for (int k = 0; k < (int)(sizeof(v.c) / sizeof(v.c[0])); ++k) v.c[k] *= s;
  }
};
template <int BS, typename Ag, typename R> struct AccL {
  R* p;
  static constexpr int NG = sizeof(Ag::c) / sizeof(R);
  __device__ __forceinline__ Ag get() const {
    Ag v;
#pragma unroll
    for (int k = 0; k < NG; ++k) v.c[k] = p[k * BS];
    return v;
  }
  __device__ __forceinline__ void set(const Ag& x) {
#pragma unroll
    for (int k = 0; k < NG; ++k) p[k * BS] = x.c[k];
  }
  __device__ __forceinline__ void add(R s, const Ag& x) {
#pragma unroll
    for (int k = 0; k < NG; ++k) p[k * BS] = fmx(s, x.c[k], p[k * BS]);
  }
  __device__ __forceinline__ void scale(R s) {
#pragma unroll
    for (int k = 0; k < NG; ++k) p[k * BS] *= s;
  }
};
template <typename R> __device__ __forceinline__ R link_token(const M3<R>& m) { return m.re[2][2]; }
template <typename R> __device__ __forceinline__ R link_token(const Q2<R>& m) { return m.q[3]; }
template <typename A> __device__ __forceinline__ A add2(const A& x, const A& y) {
  constexpr int NG = sizeof(x.c) / sizeof(x.c[0]);
  A r;
#pragma unroll
  for (int k = 0; k < NG; ++k) r.c[k] = x.c[k] + y.c[k];
  return r;
}

}  // namespace

// Layers per chunk of the march: every chunk repeats the loops of the layer before it to
// start its carries (1 / MARCH_LZ extra work) and chunks give the launch its parallelism.
#ifndef GL_MARCH_LZ
#define GL_MARCH_LZ 16
#endif
constexpr int MARCH_BS = 256;
// The five long-lived accumulators (derivatives of the site's three links, carries to two
// links of the next layer) sit in per-thread LDS slots, 5 n_g reals per thread: 80 KB per
// work-group for SU(3) in double precision, two work-groups per CU.  Held in registers
// instead, SU(3) in double precision needs about 320 registers per lane (one wave per SIMD);
// with the slots, 242 (two waves).
#ifndef GL_MARCH_CACHE
#define GL_MARCH_CACHE 1
#endif
#ifndef GL_MARCH_LDS_ACC
#define GL_MARCH_LDS_ACC 1
#endif
#ifndef GL_MARCH_WAVES
#define GL_MARCH_WAVES 2
#endif

// MarchIter (internal.h): Ebase = E(t - dt/2) + dt f1(U(t), U(t - dt)) (+ dt j on z links);
// Et the iterate E(t + dt/2), updated in place; Ut_out the new trial links exp(i a dt E') U(t);
// conv = [max |E' - E_old|, max |E'|] of this iteration (atomic max); F the MODE 0 output;
// cache (3 planes of full matrices per site): the loops of slice A alone, C_xy, C_xz^{(A,A)}
// and C_yz^{(A,A)} based at each site, which MODE 0 stores (it forms them anyway) and the
// iterations of the step read back instead of forming them (A = U(t) is fixed for the step).

bool march_geometry(const Geom& g) { return g.nt >= 8 && g.nt <= 64 && 64 % g.nt == 0; }
size_t march_cache_elems(const Geom& g, int nc) { return 3 * (size_t)(nc == 3 ? 18 : 4) * g.Vp; }

__device__ __forceinline__ void atomic_max_nn(double* addr, double v) {
  atomicMax((unsigned long long*)addr, (unsigned long long)__double_as_longlong(v));
}

template <typename G, typename T, int MODE>
__global__ void __launch_bounds__(MARCH_BS) __attribute__((amdgpu_waves_per_eu(GL_MARCH_WAVES))) k_semi_march(const T* __restrict__ A, const T* __restrict__ B, Geom g,
                                                         StepConst c, MarchIter it, int ncg, int nch) {
  using L = typename G::Link;
  using Ag = typename G::Alg;
  using R = typename G::Real;
  constexpr int NG = G::NG;
  if constexpr (MODE == 1) {
    if (it.conv_prev) {
      const double e = it.conv_prev[1];
      if (it.conv_prev[0] <= it.tol * (e > 0.0 ? e : 1e-300)) return;   // converged before
    }
  }
  const int64_t Vp = g.Vp;
  // work-group -> (chunk, column group), XCD-contiguous so that neighbouring column groups
  // (the y halo rows) of one chunk share an L2
  const uint32_t nb = (uint32_t)(ncg * nch);
  const uint32_t bid = xcd_remap(blockIdx.x, nb);
  const int cg = (int)(bid % (uint32_t)ncg), ch = (int)(bid / (uint32_t)ncg);
  const int col = cg * (MARCH_BS / 64) + (int)(threadIdx.x >> 6);
  const int ncol = (int)(g.layer / 64);
  if (col >= ncol || ch >= nch) return;   // uniform over the wavefront
  const int lane = (int)(threadIdx.x & 63u);
  const int t = col * 64 + lane;
  Site b0;
  b0.x = t % g.nt;
  b0.y = t / g.nt;
  const int z0 = ch * GL_MARCH_LZ;
  const int z1 = min(z0 + GL_MARCH_LZ, g.nz);
  const XNbr xn = x_nbr(g, b0);
  const R kxy = (R)(0.5 / (c.a[0] * c.a[0] * c.a[1] * c.a[1]));
  const R kxz = (R)(0.25 / (c.a[0] * c.a[0] * c.a[2] * c.a[2]));
  const R kyz = (R)(0.25 / (c.a[1] * c.a[1] * c.a[2] * c.a[2]));
  const R h = R(0.5);
  // Every load goes through an empty asm statement on its site index that also takes a
  // token, a value of the last loop product formed: the compiler must treat it as a new
  // load (reloading a link from the caches instead of keeping it, and forming a loop twice
  // instead of keeping it, is what holds the register count down; merging identical loads
  // would undo that), and cannot issue it before that product exists (hoisting the loads
  // of all later loops to the top of the layer would hold their links live all along).
  R tok = R(0);
  // Links are addressed by byte offsets into a direction's record array: the layers are
  // whole records (nt divides 64, nt >= 8), so the offset of a site is its layer's base
  // plus an in-layer offset that only depends on (x, y), computed once per thread for the
  // site and its +y and -y rows.
  constexpr int SW = StoredWidth<L>::value;
  constexpr uint64_t RBYTES = RecShape<T, SW>::BYTES;
  const uint64_t dir_bytes = (uint64_t)Vp * SW * sizeof(T);
  const uint64_t layer_bytes = (uint64_t)(g.layer / 64) * RBYTES;
  auto in_layer = [&](int dy) __attribute__((always_inline)) {
    const uint32_t tt = (uint32_t)(wrap_add(b0.y, dy, g.nt) * g.nt + b0.x);
    return (uint64_t)(tt / 64) * RBYTES + (uint64_t)(tt % 64) * 16;
  };
  const uint64_t o_t = in_layer(0), o_py = in_layer(1), o_my = in_layer(-1);
  const int tmy = wrap_add(b0.y, -1, g.nt) * g.nt + b0.x;   // in-layer index of the -y neighbour
  auto ld = [&](L& l, const T* U, int d, uint64_t off) __attribute__((always_inline)) {
    asm volatile("" : "+v"(off) : "v"(tok));
    using NV = typename NVec16<T>::type;
    const char* rec = (const char*)U + (uint64_t)d * dir_bytes + off;
    R v[SW];
#pragma unroll
    for (int q = 0; q < SW * (int)sizeof(T) / 16; ++q) {
      const NV x = *(const NV*)(rec + q * (RB * 16));
#pragma unroll
      for (int k = 0; k < 16 / (int)sizeof(T); ++k) v[q * (16 / (int)sizeof(T)) + k] = (R)x[k];
    }
    link_from_stored(l, v);
  };
  auto mark = [&](const L& m) __attribute__((always_inline)) { tok = link_token(m); };
  // cached loop of slice A at site index si (MODE 1), or store of a formed one (MODE 0)
  auto cached = [&](int plane, uint32_t si) __attribute__((always_inline)) -> L {
    L m;
    asm volatile("" : "+v"(si) : "v"(tok));
    load_full(m, (const T*)it.cache, plane, si, Vp);
    mark(m);
    return m;
  };
  auto keep = [&](const L& m, int plane, uint32_t si, bool warm) __attribute__((always_inline)) {
    if (GL_MARCH_CACHE && it.cache && !warm) store_full(m, (T*)it.cache, plane, si, Vp);
  };
  double dmax = 0.0, emax = 0.0;
  bool bad = false;
  // finish link d of site s with its complete derivative acc (dv/dX as components)
  auto finish = [&](const Ag& acc, int d, uint32_t s, uint64_t own) __attribute__((always_inline)) {
    const double ad = d == 0 ? c.a[0] : (d == 1 ? c.a[1] : c.a[2]);
    Ag f;
#pragma unroll
    for (int k = 0; k < NG; ++k) f.c[k] = (R)(-ad) * acc.c[k];
    if constexpr (MODE == 0) {
      store_alg(f, (T*)it.F, d, s, Vp);
    } else {
      Ag e, eo;
      load_alg_own(e, (const T*)it.Ebase, d, s, Vp);
      load_alg_own(eo, (const T*)it.Et, d, s, Vp);
      const R dt = (R)c.dt;
      const R om = (R)it.omega;
#pragma unroll
      for (int k = 0; k < NG; ++k) {
        const R en = fmx(dt, f.c[k], e.c[k]);
        dmax = fmax(dmax, fabs((double)en - (double)eo.c[k]));
        emax = fmax(emax, fabs((double)en));
        bad |= !isfinite((double)en);
        e.c[k] = fmx(om, en - eo.c[k], eo.c[k]);
      }
      store_alg(e, (T*)it.Et, d, s, Vp);
      L u;
      ld(u, A, d, own);
      store_link(G::template expi_mul<true>(e, (R)(ad * c.dt), u), (T*)it.Ut_out, d, s, Vp);
    }
  };
  // the z link at s + e_i: from the next lane for i = x, from memory for i = y
  auto zlink_i = [&](L& l, const T* U, int i, uint64_t s, uint64_t s_pi) __attribute__((always_inline)) {
    ld(l, U, 2, i == 0 ? s : s_pi);
    if (i == 0) l = pull_link(l, xn.ap);
  };
  // C^{(P,Q)}_{iz} based at s: transverse links of slice P, longitudinal of slice Q
  auto loop_iz = [&](const T* P, const T* Q, int i, uint64_t s, uint64_t s_pi, uint64_t s_pz) __attribute__((always_inline)) -> L {
    L a, bq;
    ld(a, P, i, s);
    zlink_i(bq, Q, i, s, s_pi);
    L m = G::mul(a, bq);
    ld(a, P, i, s_pz);
    m = G::mul_dag(m, a);
    ld(a, Q, 2, s);
    m = G::mul_dag(m, a);
    mark(m);
    return m;
  };
  // P(C^{(P,Q)}_{iz}) without forming the last product
  auto ploop_iz = [&](const T* P, const T* Q, int i, uint64_t s, uint64_t s_pi, uint64_t s_pz) __attribute__((always_inline)) -> Ag {
    L a, bq;
    ld(a, P, i, s);
    zlink_i(bq, Q, i, s, s_pi);
    L m = G::mul(a, bq);
    ld(a, P, i, s_pz);
    m = G::mul_dag(m, a);
    ld(a, Q, 2, s);
    const Ag r = G::proj_mul_dag(m, a);
    tok = r.c[0];
    return r;
  };
  // C_xy based at s on slice U (the y link at s + e_x from the next lane)
  auto loop_xy = [&](const T* U, uint64_t s, uint64_t s_py) __attribute__((always_inline)) -> L {
    L a, b;
    ld(a, U, 0, s);
    ld(b, U, 1, s);
    L m = G::mul(a, pull_link(b, xn.ap));
    ld(a, U, 0, s_py);
    m = G::mul_dag(m, a);
    m = G::mul_dag(m, b);
    mark(m);
    return m;
  };
  // P(C_xy) without forming the last product
  auto ploop_xy = [&](const T* U, uint64_t s, uint64_t s_py) __attribute__((always_inline)) -> Ag {
    L a, b;
    ld(a, U, 0, s);
    ld(b, U, 1, s);
    L m = G::mul(a, pull_link(b, xn.ap));
    ld(a, U, 0, s_py);
    m = G::mul_dag(m, a);
    const Ag r = G::proj_mul_dag(m, b);
    tok = r.c[0];
    return r;
  };
  // The work of a layer is a sequence of micro-steps, each forming one loop and handing its
  // derivative on; each micro-step is its own basic block (a loop that is not unrolled over
  // a switch on a uniform step number), so only the accumulators and at most two
  // projections live across them and the instruction scheduler cannot interleave loops.
  //   fx, fy, fz: derivative of the site's x, y, z links; cx, cy: carries to the x, y links
  //   of the next layer; P1, P2: projections held between the steps of one plane; snd: the
  //   (x, z) loops' derivative for the z link at s + e_x, pulled by the next lane.
  // Micro-steps 4-6 and 10-12 also serve the warm-up (the carries from the layer before the
  // chunk), where their other outputs are discarded.
#if GL_MARCH_LDS_ACC
  __shared__ R acc_lds[5 * NG * MARCH_BS];
  using A_ = AccL<MARCH_BS, Ag, R>;
  A_ fx{acc_lds + 0 * NG * MARCH_BS + threadIdx.x}, fy{acc_lds + 1 * NG * MARCH_BS + threadIdx.x},
      fz{acc_lds + 2 * NG * MARCH_BS + threadIdx.x}, cx{acc_lds + 3 * NG * MARCH_BS + threadIdx.x},
      cy{acc_lds + 4 * NG * MARCH_BS + threadIdx.x};
#else
  using A_ = Acc<Ag, R, false>;
  A_ fx, fy, fz, cx, cy;
#endif
  fx.set(G::alg_zero());
  fy.set(G::alg_zero());
  fz.set(G::alg_zero());
  cx.set(G::alg_zero());
  cy.set(G::alg_zero());
  Ag P1 = G::alg_zero(), P2 = G::alg_zero(), snd = G::alg_zero();
  constexpr int NSUB = 21, NWARM = 6;
  const int zm = z0 > 0 ? z0 - 1 : g.nz - 1;
  const int nq = NWARM + (z1 - z0) * NSUB;
#pragma unroll 1
  for (int q = 0; q < nq; ++q) {
    int z, sub;
    if (q < NWARM) {
      z = zm;
      sub = q < 3 ? 4 + q : 7 + q;
    } else {
      z = z0 + (q - NWARM) / NSUB;
      sub = (q - NWARM) % NSUB;
    }
    const int zp = z + 1 < g.nz ? z + 1 : 0;
    // byte offsets of the site, its +y and -y neighbours, and the two at z + 1
    const uint64_t lz = (uint64_t)z * layer_bytes, lzp = (uint64_t)zp * layer_bytes;
    const uint64_t s = lz + o_t, s_py = lz + o_py, s_my = lz + o_my, s_pz = lzp + o_t, s_mypz = lzp + o_my;
    const uint32_t site_z = (uint32_t)z * (uint32_t)g.layer + (uint32_t)t;   // site index (E, Et, outputs)
    const uint32_t site_my = site_z - (uint32_t)t + (uint32_t)tmy;          // its -y neighbour
    const bool warm = q < NWARM;
    L u;
    switch (sub) {
      // ---- (x, y) plane at the base: x link factor 0, y link factor 3, y link at s + e_x factor 1
      case 0:
        fx.set(cx.get());
        fy.set(cy.get());
        fz.set(G::alg_zero());
        P1 = ploop_xy(B, s, s_py);
        break;
      case 1: {
        const L CA = (MODE == 1 && GL_MARCH_CACHE) ? cached(0, site_z) : loop_xy(A, s, s_py);
        if constexpr (MODE == 0) keep(CA, 0, site_z, warm);
        const Ag hf = hs_herm<false>(CA, P1);
        fx.add(h * kxy, hf);
        fy.add(-h * kxy, hs_herm<true>(CA, P1));
        ld(u, A, 0, s);
        fy.add(h * kxy, pull_alg(G::transport(u, hf), xn.am));
        break;
      }
      // ---- (x, y) plane at base - e_y: the x link is its factor 2 (daggered), W = C F3
      case 2:
        P1 = ploop_xy(B, s_my, s);
        break;
      case 3: {
        const L CA = (MODE == 1 && GL_MARCH_CACHE) ? cached(0, site_my) : loop_xy(A, s_my, s);
        ld(u, A, 1, s_my);
        fx.add(-h * kxy, G::transport(u, hs_herm<true>(CA, P1)));
        break;
      }
      // ---- (x, z) plane at the base: x link factor 0, z link factor 3, x link at s + e_z
      // factor 2 (carry), z link at s + e_x factor 1 (snd)
      case 4:
        P1 = ploop_iz(A, B, 0, s, s, s_pz);
        break;
      case 5: {
        const L Caa = (MODE == 1 && GL_MARCH_CACHE) ? cached(1, site_z) : loop_iz(A, A, 0, s, s, s_pz);
        if constexpr (MODE == 0) keep(Caa, 1, site_z, warm);
        P2 = G::proj(Caa);
        const Ag h1 = hs_herm<false>(Caa, P1);
        const Ag hb1 = hs_herm<true>(Caa, P1);
        fx.add(h * kxz, h1);
        fz.add(-h * kxz, hb1);
        ld(u, A, 2, s);
        cx.set(G::transport(u, hb1));
        ld(u, A, 0, s);
        snd = G::transport(u, h1);
        break;
      }
      case 6: {
        const L Cab = loop_iz(A, B, 0, s, s, s_pz);
        fx.add(h * kxz, hs_herm<false>(Cab, P2));
        ld(u, B, 2, s);
        cx.add(R(1), G::transport(u, hs_herm<true>(Cab, P2)));
        cx.scale(-h * kxz);
        break;
      }
      case 7:
        P1 = ploop_iz(B, B, 0, s, s, s_pz);
        break;
      case 8: {
        const L Cba = loop_iz(B, A, 0, s, s, s_pz);
        fz.add(-h * kxz, hs_herm<true>(Cba, P1));
        ld(u, B, 0, s);
        axpy(snd, R(1), G::transport(u, hs_herm<false>(Cba, P1)));
        fz.add(h * kxz, pull_alg(snd, xn.am));
        break;
      }
      case 9:
        finish(fx.get(), 0, site_z, s);   // the x link is complete
        break;
      // ---- (y, z) plane at the base: y link factor 0, z link factor 3, y link at s + e_z
      // factor 2 (carry); its factor 1 (z link at s + e_y) is formed by the site above
      case 10:
        P1 = ploop_iz(A, B, 1, s, s_py, s_pz);
        break;
      case 11: {
        const L Caa = (MODE == 1 && GL_MARCH_CACHE) ? cached(2, site_z) : loop_iz(A, A, 1, s, s_py, s_pz);
        if constexpr (MODE == 0) keep(Caa, 2, site_z, warm);
        P2 = G::proj(Caa);
        const Ag hb1 = hs_herm<true>(Caa, P1);
        fy.add(h * kyz, hs_herm<false>(Caa, P1));
        fz.add(-h * kyz, hb1);
        ld(u, A, 2, s);
        cy.set(G::transport(u, hb1));
        break;
      }
      case 12: {
        const L Cab = loop_iz(A, B, 1, s, s_py, s_pz);
        fy.add(h * kyz, hs_herm<false>(Cab, P2));
        ld(u, B, 2, s);
        cy.add(R(1), G::transport(u, hs_herm<true>(Cab, P2)));
        cy.scale(-h * kyz);
        break;
      }
      case 13:
        P1 = ploop_iz(B, B, 1, s, s_py, s_pz);
        break;
      case 14: {
        const L Cba = loop_iz(B, A, 1, s, s_py, s_pz);
        fz.add(-h * kyz, hs_herm<true>(Cba, P1));
        break;
      }
      case 15:
        finish(fy.get(), 1, site_z, s);   // the y link is complete
        break;
      // ---- (y, z) plane at base - e_y: the z link is its factor 1, W = F0 (the y link at s - e_y)
      case 16:
        P1 = ploop_iz(A, B, 1, s_my, s, s_mypz);
        break;
      case 17: {
        const L Caa = (MODE == 1 && GL_MARCH_CACHE) ? cached(2, site_my) : loop_iz(A, A, 1, s_my, s, s_mypz);
        ld(u, A, 1, s_my);
        fz.add(h * kyz, G::transport(u, hs_herm<false>(Caa, P1)));
        break;
      }
      case 18:
        P1 = ploop_iz(B, B, 1, s_my, s, s_mypz);
        break;
      case 19: {
        const L Cba = loop_iz(B, A, 1, s_my, s, s_mypz);
        ld(u, B, 1, s_my);
        fz.add(h * kyz, G::transport(u, hs_herm<false>(Cba, P1)));
        break;
      }
      default:
        finish(fz.get(), 2, site_z, s);   // the z link is complete
        break;
    }
  }
  if constexpr (MODE == 1) {
    if (bad) dmax = INFINITY;
    for (int o = 32; o > 0; o >>= 1) {
      dmax = fmax(dmax, __shfl_down(dmax, o, 64));
      emax = fmax(emax, __shfl_down(emax, o, 64));
    }
    if (lane == 0) {
      atomic_max_nn(it.conv, dmax);
      atomic_max_nn(it.conv + 1, emax);
    }
  }
}

template <typename G, typename T>
void launch_semi_march(const T* A, const T* B, const Geom& g, const StepConst& c, int mode, const MarchIter& it,
                       hipStream_t st) {
  const int ncol = (int)(g.layer / 64);
  const int ncg = (ncol + MARCH_BS / 64 - 1) / (MARCH_BS / 64);
  const int nch = (g.nz + GL_MARCH_LZ - 1) / GL_MARCH_LZ;
  const dim3 grid((unsigned)(ncg * nch));
  if (mode == 0)
    hipLaunchKernelGGL((k_semi_march<G, T, 0>), grid, dim3(MARCH_BS), 0, st, A, B, g, c, it, ncg, nch);
  else
    hipLaunchKernelGGL((k_semi_march<G, T, 1>), grid, dim3(MARCH_BS), 0, st, A, B, g, c, it, ncg, nch);
}

#define GL_MARCH_INST(G, T) \
  template void launch_semi_march<G, T>(const T*, const T*, const Geom&, const StepConst&, int, const MarchIter&, \
                                        hipStream_t);
GL_MARCH_INST(Su2<double>, double)
GL_MARCH_INST(Su3<double>, double)
GL_MARCH_INST(Su2<float>, float)
GL_MARCH_INST(Su3<float>, float)

}  // namespace gl
