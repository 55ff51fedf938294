// Group helpers of the reverse-mode (adjoint) kernels, double precision, host + device.
// Hermitian matrices H enter products in the form i H: SU(2) a pure quaternion, SU(3) an
// anti-hermitian 3x3 matrix; G::proj of such a product returns the components of its
// hermitian part.
#pragma once
#include "group.h"

namespace gl {

template <typename G> struct AdjOps;
template <> struct AdjOps<Su2<double>> {
  using G = Su2<double>;
  // i X as a pure quaternion
  static GL_HD G::Link anti(const G::Alg& x) { return G::alg_as_link(x); }
};
template <> struct AdjOps<Su3<double>> {
  using G = Su3<double>;
  static GL_HD G::Link anti(const G::Alg& x) {
    G::Link h = G::herm(x, 1.0), r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) { r.re[i][j] = -h.im[i][j]; r.im[i][j] = h.re[i][j]; }
    return r;
  }
};

template <typename G> GL_HD typename G::Link commut(const typename G::Link& a, const typename G::Link& b) {
  typename G::Link r = G::mul(a, b);
  G::add_to(r, G::mul(b, a), -1.0);
  return r;
}

template <typename A> GL_HD void axpy(A& y, double s, const A& x) {
  constexpr int NG = sizeof(y.c) / sizeof(y.c[0]);
#pragma unroll
  for (int k = 0; k < NG; ++k) y.c[k] += s * x.c[k];
}

// c int_0^1 exp(-i s c E) Lam exp(i s c E) ds for hermitian E, Lam (components): the series
// sum_k (-ad_B)^k Lam / (k+1)!, B = i c E / 2^m with |ad_B| <= rho <= 1/2, then m doublings
// I(2B) = (I(B) + e^-B I(B) e^B) / 2.  The series stops after the fewest terms N whose
// tail bound rho^(N+1) / (N+2)! is below 2^-15 / 16! (the bound of 14 terms at rho = 1/2),
// so the truncation error is below 2^-15 / 16! relative for every field; small fields
// (rho ~ 0.02-0.1) need 7-10 terms.
template <typename G>
GL_HD typename G::Alg dexp_transpose(const typename G::Alg& e, double c, const typename G::Alg& lam) {
  using L = typename G::Link;
  constexpr int NG = G::NG;
  double n2 = 0.0;
#pragma unroll
  for (int k = 0; k < NG; ++k) n2 += e.c[k] * e.c[k];
  const double r = fabs(c) * sqrt(0.5 * n2);   // Frobenius norm of c E >= spectral norm
  int m = 0;
  double sc = 1.0;
  while (2.0 * r * sc > 0.5 && m < 60) { sc *= 0.5; ++m; }
  typename G::Alg be;
#pragma unroll
  for (int k = 0; k < NG; ++k) be.c[k] = c * sc * e.c[k];
  const L B = AdjOps<G>::anti(be);
  const L lh = AdjOps<G>::anti(lam);
  const double rho = 2.0 * r * sc;                             // bound on |ad_B|
  const double tail_max = 3.0517578125e-05 / 20922789888000.0;   // 2^-15 / 16!
  int nt = 1;
  double tail = rho * rho / 6.0;                               // rho^(N+1) / (N+2)! at N = 1
  while (nt < 14 && tail > tail_max) {
    ++nt;
    tail *= rho / (double)(nt + 2);
  }
  L T = lh;
#pragma unroll 1
  for (int k = nt; k >= 1; --k) {
    const L ad = commut<G>(B, T);
    T = lh;
    G::add_to(T, ad, -1.0 / (double)(k + 1));
  }
  if (m > 0) {
    L X = G::expi(e, -c * sc);   // exp(-B)
#pragma unroll 1
    for (int q = 0; q < m; ++q) {
      L Y = G::mul_dag(G::mul(X, T), X);   // e^-B T e^B
      G::add_to(Y, T, 1.0);
      T = G::zero();
      G::add_to(T, Y, 0.5);
      X = G::mul(X, X);
    }
  }
  typename G::Alg out = G::proj(T);
#pragma unroll
  for (int k = 0; k < NG; ++k) out.c[k] *= c;
  return out;
}

}  // namespace gl
