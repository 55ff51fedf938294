// Boost-invariant Glasma at tau = 0+ (Sec. 2, eqs. glasma_ic1, glasma_ic2, LC_gauge1): the
// longitudinal fields that infinitely thin nuclei leave at the boundary of the forward
// light cone, from the Wilson lines behind each nucleus.  With hermitian algebra
// elements and g = 1 (sum over i = x, y):
//   E_z = -i [alpha_A^i, alpha_B^i],   B_z = -i ([alpha_A^x, alpha_B^y] - [alpha_A^y, alpha_B^x]),
// eps_0 = (E_z^2 + B_z^2) / 2 = p_T.  On the transverse lattice alpha^i_N sits on the
// link (x, x + i): alpha^i_N = P(V_N(x) V_N^dag(x + i)) / a_T, P the hermitian traceless
// part of (W - W^dag)/(2i); E_z at the site averages each commutator over the two links
// of direction i that meet there, B_z at the xy plaquette centre averages alpha^x over
// the plaquette's two x links and alpha^y over its two y links.
//
// 1. per sheet k (host loop): phi_k of both nuclei by the initial-condition DFT passes,
//    then V_N <- V_N exp(-i phi_{N,k}) (k_bi_accum; later sheets on the right);
// 2. k_bi_fields: alpha, E_z, B_z per transverse site, block sums of E_z^2, B_z^2;
// 3. k_bi_finish: transverse means (eps_0, E_z^2/2, B_z^2/2).

#include "internal.h"
#include "reduce.h"

namespace gl {

// -i [X, Y] of hermitian algebra elements, as components
template <typename G> struct Comm;
template <typename T> struct Comm<Su2<T>> {
  // T^a = sigma^a / 2: -i [X, Y] = (X x Y)^a T^a
  static GL_HD Alg2<T> of(const Alg2<T>& x, const Alg2<T>& y) {
    Alg2<T> r;
    r.c[0] = x.c[1] * y.c[2] - x.c[2] * y.c[1];
    r.c[1] = x.c[2] * y.c[0] - x.c[0] * y.c[2];
    r.c[2] = x.c[0] * y.c[1] - x.c[1] * y.c[0];
    return r;
  }
};
template <typename T> struct Comm<Su3<T>> {
  // (XY - YX)/(2i) = -i [X, Y] / 2 is already hermitian traceless: -i [X, Y] = 2 P(X Y)
  static GL_HD Alg3<T> of(const Alg3<T>& x, const Alg3<T>& y) {
    Alg3<T> r = Su3<T>::proj_mul(Su3<T>::herm(x, T(1)), Su3<T>::herm(y, T(1)));
    for (int k = 0; k < 8; ++k) r.c[k] *= T(2);
    return r;
  }
};

template <typename A> GL_HD A scaled_sum(const A& x, const A& y, double s) {
  A r;
  constexpr int NG = sizeof(x.c) / sizeof(x.c[0]);
  for (int k = 0; k < NG; ++k) r.c[k] = s * (x.c[k] + y.c[k]);
  return r;
}

size_t bi_work_doubles(const Geom& g, int ng, size_t link_doubles) {
  const size_t nb = (size_t)((g.layer + 255) / 256);
  return ic_work_doubles(g, ng) + 2 * (size_t)g.layer * link_doubles + nb * NQ + 8;
}

// V_N(t) <- V_N(t) exp(-i phi_N(t)) (first: V_N(t) = exp(-i phi_N(t))), both nuclei
template <typename Gd>
__global__ void k_bi_accum(const double* __restrict__ phi, typename Gd::Link* __restrict__ V, int64_t layer,
                           int first) {
  constexpr int NG = Gd::NG;
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= 2 * layer) return;
  const int nucleus = (int)(id / layer);
  const int64_t t = id % layer;
  typename Gd::Alg p;
  for (int k = 0; k < NG; ++k) p.c[k] = phi[((int64_t)nucleus * NG + k) * layer + t];
  const typename Gd::Link e = Gd::expi(p, -1.0);
  V[id] = first ? e : Gd::mul(V[id], e);
}

template <typename Gd>
__device__ typename Gd::Alg bi_alpha(const typename Gd::Link* __restrict__ V, int nt, int x, int y, int i,
                                     double inv_aT) {
  const int xp = i == 0 ? wrap_add(x, 1, nt) : x;
  const int yp = i == 1 ? wrap_add(y, 1, nt) : y;
  typename Gd::Alg a = Gd::proj_mul_dag(V[(int64_t)y * nt + x], V[(int64_t)yp * nt + xp]);
  constexpr int NG = Gd::NG;
  for (int k = 0; k < NG; ++k) a.c[k] *= inv_aT;
  return a;
}

template <typename Gd>
__global__ void __launch_bounds__(256) k_bi_fields(const typename Gd::Link* __restrict__ V, int nt, double a_T,
                                                   double* __restrict__ Ez, double* __restrict__ Bz,
                                                   double* __restrict__ partial) {
  using A = typename Gd::Alg;
  constexpr int NG = Gd::NG;
  const int64_t layer = (int64_t)nt * nt;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double acc[NQ];
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
  if (t < layer) {
    const typename Gd::Link* VA = V;
    const typename Gd::Link* VB = V + layer;
    const int x = (int)(t % nt), y = (int)(t / nt);
    const int xm = wrap_add(x, -1, nt), ym = wrap_add(y, -1, nt);
    const int xp = wrap_add(x, 1, nt), yp = wrap_add(y, 1, nt);
    const double s = 1.0 / a_T;
    // E_z at the site: links (x, x+i) and (x-i, x) of both directions
    const A cx0 = Comm<Gd>::of(bi_alpha<Gd>(VA, nt, x, y, 0, s), bi_alpha<Gd>(VB, nt, x, y, 0, s));
    const A cx1 = Comm<Gd>::of(bi_alpha<Gd>(VA, nt, xm, y, 0, s), bi_alpha<Gd>(VB, nt, xm, y, 0, s));
    const A cy0 = Comm<Gd>::of(bi_alpha<Gd>(VA, nt, x, y, 1, s), bi_alpha<Gd>(VB, nt, x, y, 1, s));
    const A cy1 = Comm<Gd>::of(bi_alpha<Gd>(VA, nt, x, ym, 1, s), bi_alpha<Gd>(VB, nt, x, ym, 1, s));
    A ez;
    for (int k = 0; k < NG; ++k) ez.c[k] = 0.5 * (cx0.c[k] + cx1.c[k]) + 0.5 * (cy0.c[k] + cy1.c[k]);
    // B_z at the plaquette (x, x+x, x+x+y, x+y)
    const A axA = scaled_sum(bi_alpha<Gd>(VA, nt, x, y, 0, s), bi_alpha<Gd>(VA, nt, x, yp, 0, s), 0.5);
    const A axB = scaled_sum(bi_alpha<Gd>(VB, nt, x, y, 0, s), bi_alpha<Gd>(VB, nt, x, yp, 0, s), 0.5);
    const A ayA = scaled_sum(bi_alpha<Gd>(VA, nt, x, y, 1, s), bi_alpha<Gd>(VA, nt, xp, y, 1, s), 0.5);
    const A ayB = scaled_sum(bi_alpha<Gd>(VB, nt, x, y, 1, s), bi_alpha<Gd>(VB, nt, xp, y, 1, s), 0.5);
    const A b1 = Comm<Gd>::of(axA, ayB), b2 = Comm<Gd>::of(ayA, axB);
    A bz;
    for (int k = 0; k < NG; ++k) bz.c[k] = b1.c[k] - b2.c[k];
    for (int k = 0; k < NG; ++k) {
      Ez[(int64_t)k * layer + t] = ez.c[k];
      Bz[(int64_t)k * layer + t] = bz.c[k];
    }
    acc[0] = norm2(ez);
    acc[1] = norm2(bz);
  }
  block_reduce_write<256>(acc, 3u, partial + (int64_t)blockIdx.x * NQ);
}

__global__ void k_bi_finish(const double* __restrict__ partial, int nb, int64_t layer, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double e = 0.0, b = 0.0;
  for (int k = 0; k < nb; ++k) {
    e += partial[(int64_t)k * NQ + 0];
    b += partial[(int64_t)k * NQ + 1];
  }
  e *= 0.5 / (double)layer;
  b *= 0.5 / (double)layer;
  out[0] = e + b;
  out[1] = e;
  out[2] = b;
}

template <int NC>
void launch_bi_sheet(const double* phi, double* work_links, const Geom& g, int first, hipStream_t st) {
  using Gd = typename GroupOf<NC, double>::type;
  const int64_t n = 2 * g.layer;
  hipLaunchKernelGGL((k_bi_accum<Gd>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, phi,
                     (typename Gd::Link*)work_links, g.layer, first);
}

template <int NC>
void launch_bi_fields(const double* work_links, double* partial, const Geom& g, double a_T, double* Ez, double* Bz,
                      double* out3, hipStream_t st) {
  using Gd = typename GroupOf<NC, double>::type;
  const int nb = (int)((g.layer + 255) / 256);
  hipLaunchKernelGGL((k_bi_fields<Gd>), dim3(nb), dim3(256), 0, st, (const typename Gd::Link*)work_links, g.nt,
                     a_T, Ez, Bz, partial);
  hipLaunchKernelGGL(k_bi_finish, dim3(1), dim3(64), 0, st, partial, nb, g.layer, out3);
}

template void launch_bi_sheet<2>(const double*, double*, const Geom&, int, hipStream_t);
template void launch_bi_sheet<3>(const double*, double*, const Geom&, int, hipStream_t);
template void launch_bi_fields<2>(const double*, double*, const Geom&, double, double*, double*, double*, hipStream_t);
template void launch_bi_fields<3>(const double*, double*, const Geom&, double, double*, double*, double*, hipStream_t);

}  // namespace gl
