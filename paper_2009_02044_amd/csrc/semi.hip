// Semi-implicit scheme with time-averaged plaquette-like terms (Sec. 3, fig. wilson and
// the text on the numerical Cherenkov instability; Sec. 5): the reading implemented
// here replaces the Wilson potential of one time slice by a potential between two
// neighbouring slices m, m+1 (X.Y = sum_a X^a Y^a)
//   v(m, m+1) = k_xy P(C_xy^m) . P(C_xy^{m+1})
//             + sum_{i=x,y} k_iz [ P(C_iz^{(m,m)}) . P(C_iz^{(m,m+1)}) + P(C_iz^{(m+1,m+1)}) . P(C_iz^{(m+1,m)}) ],
//   k_xy = 1/(2 a_x^2 a_y^2), k_iz = 1/(4 a_i^2 a_z^2),
// where C_iz^{(m,m')} is the (i, z) plaquette with its transverse links on slice m and
// its longitudinal links on slice m'.  v is symmetric in the two slices, so with
// f1(A, B) = -a_d dv(A, B)/dX (left variation U -> exp(iX) U of a slice-A link) the
// force at time t is F = f1(U(t), U(t-dt)) + f1(U(t), U(t+dt)), and the step
//   E(t+dt/2) = E(t-dt/2) + dt (F + j),  U(t+dt) = exp(i a dt E(t+dt/2)) U(t)
// is solved by fixed-point iteration on E(t+dt/2); U(t-dt) = exp(-i a dt E(t-dt/2)) U(t).
//
// Derivative rule: for a term 2 Tr(P(C) Y) with C = F0 F1 F2 F3 based at b and
// H = C Y + Y C^dag, a non-daggered factor k contributes +1/2 W^dag H W with W the
// product of the factors before it, a daggered factor -1/2 W^dag H W with W the product
// up to and including it, at the factor's own link.  For k = 3 (W = C) this is
// -1/2 (Y C + C^dag Y); for the daggered k = 2 factor W = C F3.
#include "internal.h"
#include "stencil.h"

namespace gl {

// C_xy(b) = U_x(b) U_y(b+x) U_x^dag(b+y) U_y^dag(b) on one slice
template <typename G, typename T>
__device__ __forceinline__ typename G::Link loop_xy(const T* __restrict__ U, const Geom& g, Site b) {
  using L = typename G::Link;
  const int64_t Vp = g.Vp;
  L a, bb, c, d;
  load_link(a, U, 0, idx(g, b), Vp);
  load_link(bb, U, 1, idx(g, shifted(g, b, 0, 1)), Vp);
  load_link(c, U, 0, idx(g, shifted(g, b, 1, 1)), Vp);
  load_link(d, U, 1, idx(g, b), Vp);
  return G::mul_dag(G::mul_dag(G::mul(a, bb), c), d);
}

// C_iz(b) = U_i(b) U_z(b+i) U_i^dag(b+z) U_z^dag(b), transverse links from Ui, longitudinal from Uz
template <typename G, typename T>
__device__ __forceinline__ typename G::Link loop_iz(const T* __restrict__ Ui, const T* __restrict__ Uz,
                                                    const Geom& g, Site b, int i) {
  using L = typename G::Link;
  const int64_t Vp = g.Vp;
  L a, bb, c, d;
  load_link(a, Ui, i, idx(g, b), Vp);
  load_link(bb, Uz, 2, idx(g, shifted(g, b, i, 1)), Vp);
  load_link(c, Ui, i, idx(g, shifted(g, b, 2, 1)), Vp);
  load_link(d, Uz, 2, idx(g, b), Vp);
  return G::mul_dag(G::mul_dag(G::mul(a, bb), c), d);
}

template <typename G>
__device__ __forceinline__ typename G::Link herm_P(const typename G::Link& C) {
  return G::herm_from_alg(G::proj(C));
}
// M + M^dag for a product M of a loop and a hermitian Y.  SU(3) carries a hermitian X as X
// itself; SU(2) carries it as i X (a quaternion), where the same sum reads M - M^dag.
template <typename G>
__device__ __forceinline__ typename G::Link herm_sum(const typename G::Link& m) {
  typename G::Link h = m;
  G::add_to(h, G::dag(m), (typename G::Real)(G::NC == 3 ? 1 : -1));
  return h;
}
// C Y + Y C^dag = M + M^dag with M = C Y (Y hermitian): one product instead of two
template <typename G>
__device__ __forceinline__ typename G::Link Hf(const typename G::Link& C, const typename G::Link& Y) {
  return herm_sum<G>(G::mul(C, Y));
}
// Y C + C^dag Y  (= C^dag H C) = N + N^dag with N = Y C
template <typename G>
__device__ __forceinline__ typename G::Link Hb(const typename G::Link& C, const typename G::Link& Y) {
  return herm_sum<G>(G::mul(Y, C));
}
// W^dag X W
template <typename G>
__device__ __forceinline__ typename G::Link conj_by(const typename G::Link& W, const typename G::Link& X) {
  return G::dag_mul(W, G::mul(X, W));
}

// f1(A, B) for the link (y, d) of slice A: returns -a_d dv(A, B)/dX as components.  The
// direction is a template argument: each direction's kernel holds only its own terms.
template <typename G, typename T, int d>
__device__ typename G::Alg semi_f1(const T* __restrict__ A, const T* __restrict__ B, const Geom& g, Site y,
                                   const StepConst& c) {
  using L = typename G::Link;
  using R = typename G::Real;
  const int64_t Vp = g.Vp;
  L acc = G::zero();
  if constexpr (d < 2) {
    // (x, y) plane: loop C_xy[A] with Y = P(C_xy[B]) at the same base
    const R kxy = (R)(0.5 / (c.a[0] * c.a[0] * c.a[1] * c.a[1]));
    if constexpr (d == 0) {
      {  // factor 0 at base y: +1/2 H
        L C = loop_xy<G, T>(A, g, y), Y = herm_P<G>(loop_xy<G, T>(B, g, y));
        G::add_to(acc, Hf<G>(C, Y), R(0.5) * kxy);
      }
      {  // factor 2 (daggered) at base y - y^: -1/2 F3^dag (Y C + C^dag Y) F3, F3 = U_y(b)
        Site b = shifted(g, y, 1, -1);
        L C = loop_xy<G, T>(A, g, b), Y = herm_P<G>(loop_xy<G, T>(B, g, b));
        L F3;
        load_link(F3, A, 1, idx(g, b), Vp);
        G::add_to(acc, conj_by<G>(F3, Hb<G>(C, Y)), R(-0.5) * kxy);
      }
    } else {
      {  // factor 1 at base y - x^: +1/2 F0^dag H F0, F0 = U_x(b)
        Site b = shifted(g, y, 0, -1);
        L C = loop_xy<G, T>(A, g, b), Y = herm_P<G>(loop_xy<G, T>(B, g, b));
        L F0;
        load_link(F0, A, 0, idx(g, b), Vp);
        G::add_to(acc, conj_by<G>(F0, Hf<G>(C, Y)), R(0.5) * kxy);
      }
      {  // factor 3 (daggered) at base y: -1/2 (Y C + C^dag Y)
        L C = loop_xy<G, T>(A, g, y), Y = herm_P<G>(loop_xy<G, T>(B, g, y));
        G::add_to(acc, Hb<G>(C, Y), R(-0.5) * kxy);
      }
    }
    // (d, z) plane: C_AA = C^{(A,A)}, C_AB = C^{(A,B)}; both carry this link as factors 0 and 2
    const R kiz = (R)(0.25 / (c.a[d] * c.a[d] * c.a[2] * c.a[2]));
    {  // base y, factor 0: +1/2 [H(C_AA, P_AB) + H(C_AB, P_AA)]
      L Caa = loop_iz<G, T>(A, A, g, y, d), Cab = loop_iz<G, T>(A, B, g, y, d);
      L Paa = herm_P<G>(Caa), Pab = herm_P<G>(Cab);
      L h = Hf<G>(Caa, Pab);
      G::add_to(h, Hf<G>(Cab, Paa), R(1));
      G::add_to(acc, h, R(0.5) * kiz);
    }
    {  // base y - z^, factor 2 (daggered): -1/2 [F3a^dag Hb(C_AA, P_AB) F3a + F3b^dag Hb(C_AB, P_AA) F3b]
      Site b = shifted(g, y, 2, -1);
      L Caa = loop_iz<G, T>(A, A, g, b, d), Cab = loop_iz<G, T>(A, B, g, b, d);
      L Paa = herm_P<G>(Caa), Pab = herm_P<G>(Cab);
      L Fa, Fb;
      load_link(Fa, A, 2, idx(g, b), Vp);
      load_link(Fb, B, 2, idx(g, b), Vp);
      L h = conj_by<G>(Fa, Hb<G>(Caa, Pab));
      G::add_to(h, conj_by<G>(Fb, Hb<G>(Cab, Paa)), R(1));
      G::add_to(acc, h, R(-0.5) * kiz);
    }
  } else {
    // longitudinal link: planes (x, z) and (y, z); loops with z links on slice A:
    // C_AA (Y = P(C_AB)) and C_BA (Y = P(C_BB)); the link is factor 1 at base y - i^
    // and factor 3 (daggered) at base y
#pragma unroll 1
    for (int i = 0; i < 2; ++i) {
      const R kiz = (R)(0.25 / (c.a[i] * c.a[i] * c.a[2] * c.a[2]));
      {
        Site b = shifted(g, y, i, -1);
        L Caa = loop_iz<G, T>(A, A, g, b, i), Cab = loop_iz<G, T>(A, B, g, b, i);
        L Cba = loop_iz<G, T>(B, A, g, b, i), Cbb = loop_iz<G, T>(B, B, g, b, i);
        L Fa, Fb;
        load_link(Fa, A, i, idx(g, b), Vp);
        load_link(Fb, B, i, idx(g, b), Vp);
        L h = conj_by<G>(Fa, Hf<G>(Caa, herm_P<G>(Cab)));
        G::add_to(h, conj_by<G>(Fb, Hf<G>(Cba, herm_P<G>(Cbb))), R(1));
        G::add_to(acc, h, R(0.5) * kiz);
      }
      {
        L Caa = loop_iz<G, T>(A, A, g, y, i), Cab = loop_iz<G, T>(A, B, g, y, i);
        L Cba = loop_iz<G, T>(B, A, g, y, i), Cbb = loop_iz<G, T>(B, B, g, y, i);
        L h = Hb<G>(Caa, herm_P<G>(Cab));
        G::add_to(h, Hb<G>(Cba, herm_P<G>(Cbb)), R(1));
        G::add_to(acc, h, R(-0.5) * kiz);
      }
    }
  }
  typename G::Alg f = G::alg_from_herm(acc);
  const R ka = (R)(-c.a[d]);
#pragma unroll
  for (int k = 0; k < G::NG; ++k) f.c[k] *= ka;
  return f;
}

template <typename G>
__device__ __forceinline__ void site_of(const Geom& g, uint32_t s, Site& x) {
  x.x = (int)(s % (uint32_t)g.nt);
  x.y = (int)((s / (uint32_t)g.nt) % (uint32_t)g.nt);
  x.z = (int)(s / (uint32_t)g.layer);
}

// out = f1(Uc, Uo) for every link of direction d
template <typename G, typename T, int d>
__global__ void __launch_bounds__(256) k_semi_f1(const T* __restrict__ Uc, const T* __restrict__ Uo,
                                                 T* __restrict__ out, Geom g, StepConst c) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= (uint32_t)g.V) return;
  Site x;
  site_of<G>(g, s, x);
  typename G::Alg f = semi_f1<G, T, d>(Uc, Uo, g, x, c);
  store_alg(f, out, d, s, g.Vp);
}

// U(t-dt) = exp(-i a dt E) U(t) into Up, first trial U(t+dt) = exp(+i a dt E) U(t) into Ut,
// first trial E(t+dt/2) into Et and U(t+dt) = exp(+i a dt Et) U(t) into Ut.  With the
// previous step at hand, Ep = E(t-3dt/2) + dt j(t-dt) (k_semi_keep), so E - Ep is the last
// step's field increment without its current: the trial is E + (E - Ep) + dt j(t) (the
// current of this step, J, on hop steps), else E(t-dt/2) (+ dt j).  Only the starting point
// of the iteration; its fixed point is the same.
template <typename G, typename T>
__global__ void __launch_bounds__(256) k_semi_begin(const T* __restrict__ U, const T* __restrict__ E,
                                                    const T* __restrict__ Ep, const T* __restrict__ J,
                                                    T* __restrict__ Up, T* __restrict__ Ut, T* __restrict__ Et,
                                                    Geom g, StepConst c) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= (uint32_t)g.V) return;
  const int d = blockIdx.y;
  typename G::Link u;
  typename G::Alg e, et;
  load_link(u, U, d, s, g.Vp);
  load_alg(e, E, d, s, g.Vp);
  et = e;
  if (Ep) {
    typename G::Alg ep;
    load_alg(ep, Ep, d, s, g.Vp);
#pragma unroll
    for (int k = 0; k < G::NG; ++k) et.c[k] = e.c[k] + (e.c[k] - ep.c[k]);
  }
  if (J && d == 2) {
    typename G::Alg j;
    load_alg(j, J, 0, s, g.Vp);
#pragma unroll
    for (int k = 0; k < G::NG; ++k) et.c[k] += j.c[k];
  }
  const typename G::Real k = (typename G::Real)(c.a[d] * c.dt);
  store_link(G::mul(G::expi(e, -k), u), Up, d, s, g.Vp);
  store_link(G::mul(G::expi(et, k), u), Ut, d, s, g.Vp);
  store_alg(et, Et, d, s, g.Vp);
}

// after a step: Ep = E(t-dt/2) + [z] dt j(t) (J on hop steps), the reference of the next
// step's starting guess
template <typename G, typename T>
__global__ void __launch_bounds__(256) k_semi_keep(const T* __restrict__ E, const T* __restrict__ J,
                                                   T* __restrict__ Ep, Geom g) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= (uint32_t)g.V) return;
  const int d = blockIdx.y;
  typename G::Alg e;
  load_alg(e, E, d, s, g.Vp);
  if (J && d == 2) {
    typename G::Alg j;
    load_alg(j, J, 0, s, g.Vp);
#pragma unroll
    for (int k = 0; k < G::NG; ++k) e.c[k] += j.c[k];
  }
  store_alg(e, Ep, d, s, g.Vp);
}

// The hop of both charge populations with the links U(t): COMMIT = false writes only the
// current dt j_z = a_L (rho_A' - rho_B) (the solve needs it; the charges stay where they are
// until the solve has converged), COMMIT = true moves the charges in place (J unused).
template <typename G, typename T, bool COMMIT>
__global__ void __launch_bounds__(256) k_semi_hop(const T* __restrict__ U, T* __restrict__ rhoA,
                                                  T* __restrict__ rhoB, T* __restrict__ J, Geom g, StepConst c) {
  using A = typename G::Alg;
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= (uint32_t)g.V) return;
  Site x;
  site_of<G>(g, s, x);
  const int64_t Vp = g.Vp;
  typename G::Link Uz;
  load_link(Uz, U, 2, s, Vp);
  const uint32_t sB = site_index(g, x.x, x.y, slotB(x.z, c.offB, g.nz));
  const uint32_t sA = site_index(g, x.x, x.y, slotA(wrap_add(x.z, 1, g.nz), c.offA, g.nz));
  A rb, ra;
  load_alg_own(rb, rhoB, 0, sB, Vp);
  load_alg_own(ra, rhoA, 0, sA, Vp);
  A ran = G::transport_inv(Uz, ra);
  if constexpr (COMMIT) {
    store_alg(G::transport(Uz, rb), rhoB, 0, sB, Vp);
    store_alg(ran, rhoA, 0, sA, Vp);
  } else {
    A jz;
    const typename G::Real al = (typename G::Real)c.a[2];
#pragma unroll
    for (int k = 0; k < G::NG; ++k) jz.c[k] = al * (ran.c[k] - rb.c[k]);
    store_alg(jz, J, 0, s, Vp);
  }
}

// zero n doubles (the convergence slots of a batch of iterations; a kernel, not a memset,
// so that the sequence stays capturable)
__global__ void k_zero(double* __restrict__ p, int n) {
  const int k = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (k < n) p[k] = 0.0;
}

__device__ __forceinline__ void atomic_max_nonneg(double* addr, double v) {
  // non-negative doubles order like their bit patterns
  atomicMax((unsigned long long*)addr, (unsigned long long)__double_as_longlong(v));
}

// Convergence test of an iteration's slot: max |dE| <= tol max |E| (both 0: converged).
// A non-finite field leaves +inf in conv[0], which never passes.
__device__ __forceinline__ bool semi_converged(const double* conv, double tol) {
  const double e = conv[1];
  return conv[0] <= tol * (e > 0.0 ? e : 1e-300);
}

// One fixed-point iteration: E' = Ebase + dt f1(Uc, Ut_in) with Ebase = E + dt f1(Uc, U(t - dt))
// + [z] dt j (k_semi_base), Ut_out = exp(i a dt E') Uc, Et <- E'; conv[0] = max |E' - Et_old|
// (+inf if E' is not finite), conv[1] = max |E'| (component-wise).  When the previous
// iteration's slot conv_prev already passes the test the iteration does nothing (every
// thread returns): the host enqueues several iterations at once and reads their slots
// afterwards.  (Lattices whose rows fill wavefronts use the marching pass of semi_march.hip.)
template <typename G, typename T, int d>
__device__ __forceinline__ void semi_iter_body(const T* __restrict__ Uc, const T* __restrict__ Ut_in,
                                               const T* __restrict__ Ebase, T* __restrict__ Et,
                                               T* __restrict__ Ut_out, double* __restrict__ conv,
                                               const double* __restrict__ conv_prev, double tol, const Geom& g,
                                               const StepConst& c, double omega) {
  using A = typename G::Alg;
  if (conv_prev && semi_converged(conv_prev, tol)) return;
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  double dmax = 0.0, emax = 0.0;
  if (s < (uint32_t)g.V) {
    Site x;
    site_of<G>(g, s, x);
    const int64_t Vp = g.Vp;
    A f = semi_f1<G, T, d>(Uc, Ut_in, g, x, c);
    A e, eo;
    load_alg_own(e, Ebase, d, s, Vp);
    load_alg_own(eo, Et, d, s, Vp);
    const typename G::Real dt = (typename G::Real)c.dt;
#pragma unroll
    for (int k = 0; k < G::NG; ++k) e.c[k] = fmx(dt, f.c[k], e.c[k]);
    bool bad = false;
#pragma unroll
    for (int k = 0; k < G::NG; ++k) {
      dmax = fmax(dmax, fabs((double)e.c[k] - (double)eo.c[k]));
      emax = fmax(emax, fabs((double)e.c[k]));
      bad |= !isfinite((double)e.c[k]);
    }
    // fmax drops a NaN operand: a non-finite field is reported as an infinite update
    if (bad) dmax = INFINITY;
    // under-relaxed update of the iterate: eo + omega (E' - eo)
    const typename G::Real om = (typename G::Real)omega;
#pragma unroll
    for (int k = 0; k < G::NG; ++k) e.c[k] = fmx(om, e.c[k] - eo.c[k], eo.c[k]);
    store_alg(e, Et, d, s, Vp);
    typename G::Link u;
    load_link(u, Uc, d, s, Vp);
    store_link(G::mul(G::expi(e, (typename G::Real)(c.a[d] * c.dt)), u), Ut_out, d, s, Vp);
  }
  for (int o = 32; o > 0; o >>= 1) {
    dmax = fmax(dmax, __shfl_down(dmax, o, 64));
    emax = fmax(emax, __shfl_down(emax, o, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    atomic_max_nonneg(conv, dmax);
    atomic_max_nonneg(conv + 1, emax);
  }
}
// Transverse links: held to two waves per SIMD (a few bytes of spill, against one wave
// without the bound); the longitudinal link's terms need more registers than that allows.
template <typename G, typename T, int d>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_semi_iter_t(const T* __restrict__ Uc, const T* __restrict__ Ut_in, const T* __restrict__ Ebase,
              T* __restrict__ Et, T* __restrict__ Ut_out, double* __restrict__ conv,
              const double* __restrict__ conv_prev, double tol, Geom g, StepConst c, double omega) {
  semi_iter_body<G, T, d>(Uc, Ut_in, Ebase, Et, Ut_out, conv, conv_prev, tol, g, c, omega);
}
template <typename G, typename T>
__global__ void __launch_bounds__(256) k_semi_iter_z(const T* __restrict__ Uc, const T* __restrict__ Ut_in,
                                                     const T* __restrict__ Ebase, T* __restrict__ Et,
                                                     T* __restrict__ Ut_out, double* __restrict__ conv,
                                                     const double* __restrict__ conv_prev, double tol, Geom g,
                                                     StepConst c, double omega) {
  semi_iter_body<G, T, 2>(Uc, Ut_in, Ebase, Et, Ut_out, conv, conv_prev, tol, g, c, omega);
}

// Ebase = E(t - dt/2) + dt F2 + [z] dt j, in place over F2 (F2 = f1(U(t), U(t - dt)); J holds
// dt j_z on hop steps, else null): the part of the fixed-point map that does not change.
template <typename G, typename T>
__global__ void __launch_bounds__(256) k_semi_base(const T* __restrict__ E, T* __restrict__ F2,
                                                   const T* __restrict__ J, Geom g, double dt) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= (uint32_t)g.V) return;
  const int d = blockIdx.y;
  typename G::Alg e, f;
  load_alg_own(e, E, d, s, g.Vp);
  load_alg_own(f, F2, d, s, g.Vp);
  const typename G::Real k = (typename G::Real)dt;
#pragma unroll
  for (int q = 0; q < G::NG; ++q) e.c[q] = fmx(k, f.c[q], e.c[q]);
  if (J && d == 2) {
    typename G::Alg j;
    load_alg_own(j, J, 0, s, g.Vp);
#pragma unroll
    for (int q = 0; q < G::NG; ++q) e.c[q] += j.c[q];
  }
  store_alg(e, F2, d, s, g.Vp);
}

template <typename G, typename T>
__global__ void k_copy_alg(const T* __restrict__ src, T* __restrict__ dst, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) dst[k] = src[k];
}

template <typename G, typename T>
void launch_semi_f1(const T* Uc, const T* Uo, T* out, const Geom& g, const StepConst& c, hipStream_t st, T* cache) {
  if (march_geometry(g)) {
    MarchIter it{};
    it.F = out;
    it.cache = cache;
    launch_semi_march<G, T>(Uc, Uo, g, c, 0, it, st);
    return;
  }
  const int bs = 256;
  const dim3 grid((unsigned)((g.V + bs - 1) / bs));
  hipLaunchKernelGGL((k_semi_f1<G, T, 0>), grid, dim3(bs), 0, st, Uc, Uo, out, g, c);
  hipLaunchKernelGGL((k_semi_f1<G, T, 1>), grid, dim3(bs), 0, st, Uc, Uo, out, g, c);
  hipLaunchKernelGGL((k_semi_f1<G, T, 2>), grid, dim3(bs), 0, st, Uc, Uo, out, g, c);
}

template <typename G, typename T>
void launch_semi_base(const T* E, T* F2, const T* J, const Geom& g, double dt, hipStream_t st) {
  const int bs = 256;
  hipLaunchKernelGGL((k_semi_base<G, T>), dim3((unsigned)((g.V + bs - 1) / bs), 3), dim3(bs), 0, st, E, F2, J, g, dt);
}

template <typename G, typename T>
void launch_semi_begin(const T* U, const T* E, const T* Ep, const T* J, T* Up, T* Ut, T* Et, const Geom& g,
                       const StepConst& c, hipStream_t st) {
  const int bs = 256;
  hipLaunchKernelGGL((k_semi_begin<G, T>), dim3((unsigned)((g.V + bs - 1) / bs), 3), dim3(bs), 0, st, U, E, Ep, J,
                     Up, Ut, Et, g, c);
}

template <typename G, typename T>
void launch_semi_keep(const T* E, const T* J, T* Ep, const Geom& g, hipStream_t st) {
  const int bs = 256;
  hipLaunchKernelGGL((k_semi_keep<G, T>), dim3((unsigned)((g.V + bs - 1) / bs), 3), dim3(bs), 0, st, E, J, Ep, g);
}

template <typename G, typename T>
void launch_semi_hop(const T* U, T* rhoA, T* rhoB, T* J, bool commit, const Geom& g, const StepConst& c,
                     hipStream_t st) {
  const int bs = 256;
  const dim3 grid((unsigned)((g.V + bs - 1) / bs));
  if (commit) hipLaunchKernelGGL((k_semi_hop<G, T, true>), grid, dim3(bs), 0, st, U, rhoA, rhoB, J, g, c);
  else hipLaunchKernelGGL((k_semi_hop<G, T, false>), grid, dim3(bs), 0, st, U, rhoA, rhoB, J, g, c);
}

void launch_zero(double* p, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
}

template <typename G, typename T>
void launch_semi_iter(const T* Uc, const T* Ut_in, const T* Ebase, T* Et, T* Ut_out, double* conv,
                      const double* conv_prev, double tol, const Geom& g, const StepConst& c, hipStream_t st,
                      const T* cache) {
  const int bs = 256;
  // Under-relaxation of the fixed-point map E -> E(t-dt/2) + dt (F2 + f1(U, U(E)) + j).  Its
  // linearisation is implicit only in the slice-averaged transverse terms, with eigenvalues in
  // [-4 dt^2 / a_T^2, 0] (the spread of -dt^2 K_T / 2, K_T <= 8 / a_T^2); the relaxation
  // omega = 2 / (2 - lambda_min) = 1 / (1 + 2 dt^2 / a_T^2) minimises the spectral radius of
  // the relaxed map (0.25 -> 0.11 at dt = a_L, a_T = 4 a_L).  Same fixed point.
  const double omega = 1.0 / (1.0 + 2.0 * c.dt * c.dt / (c.a[0] * c.a[0]));
  if (march_geometry(g)) {
    MarchIter it{};
    it.Ebase = Ebase;
    it.Et = Et;
    it.Ut_out = Ut_out;
    it.conv = conv;
    it.conv_prev = conv_prev;
    it.tol = tol;
    it.omega = omega;
    it.cache = (void*)cache;
    launch_semi_march<G, T>(Uc, Ut_in, g, c, 1, it, st);
    return;
  }
  const dim3 grid((unsigned)((g.V + bs - 1) / bs));
  // one launch per direction: a kernel holds only that direction's terms
  hipLaunchKernelGGL((k_semi_iter_t<G, T, 0>), grid, dim3(bs), 0, st, Uc, Ut_in, Ebase, Et, Ut_out, conv, conv_prev,
                     tol, g, c, omega);
  hipLaunchKernelGGL((k_semi_iter_t<G, T, 1>), grid, dim3(bs), 0, st, Uc, Ut_in, Ebase, Et, Ut_out, conv, conv_prev,
                     tol, g, c, omega);
  hipLaunchKernelGGL((k_semi_iter_z<G, T>), grid, dim3(bs), 0, st, Uc, Ut_in, Ebase, Et, Ut_out, conv, conv_prev, tol,
                     g, c, omega);
}

template <typename G, typename T>
void launch_copy(const T* src, T* dst, int64_t n, hipStream_t st) {
  const int bs = 256;
  hipLaunchKernelGGL((k_copy_alg<G, T>), dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, st, src, dst, n);
}

#define GL_SEMI_INST(G, T)                                                                                      \
  template void launch_semi_f1<G, T>(const T*, const T*, T*, const Geom&, const StepConst&, hipStream_t, T*); \
  template void launch_semi_keep<G, T>(const T*, const T*, T*, const Geom&, hipStream_t);                    \
  template void launch_semi_begin<G, T>(const T*, const T*, const T*, const T*, T*, T*, T*, const Geom&,        \
                                        const StepConst&, \
                                        hipStream_t);                                                          \
  template void launch_semi_hop<G, T>(const T*, T*, T*, T*, bool, const Geom&, const StepConst&, hipStream_t); \
  template void launch_semi_iter<G, T>(const T*, const T*, const T*, T*, T*, double*, const double*, double,    \
                                       const Geom&, const StepConst&, hipStream_t, const T*);                  \
  template void launch_semi_base<G, T>(const T*, T*, const T*, const Geom&, double, hipStream_t);             \
  template void launch_copy<G, T>(const T*, T*, int64_t, hipStream_t);
GL_SEMI_INST(Su2<double>, double)
GL_SEMI_INST(Su3<double>, double)
GL_SEMI_INST(Su2<float>, float)
GL_SEMI_INST(Su3<float>, float)

}  // namespace gl
