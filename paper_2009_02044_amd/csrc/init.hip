// Initial conditions of two MV nuclei with finite longitudinal extent, computed on
// the GPU in double precision (Sec. 2: Gaussian W[rho] and the Fourier solution of
// the transverse Poisson equation with IR regulator m and UV cutoff Lambda;
// Sec. 3: eqs. single_sheet, 3d_colorfield_1, 3d_colorfield_2, the temporal gauge,
// and the CPIC charges that satisfy eq. gauss).
//
// 1. phi^a_N = DFT^-1[ rho~^a_N Theta(Lambda - |k~|) / (k~^2 + m^2) ] on the nt x nt
//    transverse torus, k~^2 = (2/a_T)^2 (sin^2(pi kx/nt) + sin^2(pi ky/nt)), by four
//    separable direct DFT passes (nt <= a few hundred, one-shot per event).
// 2. Wilson lines V_N(x, t) = exp(-i Lambda_N(z, t) phi_N(x_T)): the colour structure
//    of a single sheet does not depend on z, so the path ordering is trivial and the
//    cumulative normalised Gaussian profile is
//      Lambda_B = erfc((z - z_B - (t - t0)) / (sqrt 2 sigma)) / 2   (B moves +z),
//      Lambda_A = erfc(-(z - z_A + (t - t0)) / (sqrt 2 sigma)) / 2  (A moves -z).
//    With ns sheets (colour structure varying along the beam axis, independent
//    charges per piece of equal profile weight, Sec. 3 after eq. single_sheet and
//    Sec. 5) the line is the path-ordered product
//      V_N = exp(-i lambda_0 phi_{N,0}) ... exp(-i lambda_{ns-1} phi_{N,ns-1}),
//      lambda_k = clamp(ns Lambda_N - k, 0, 1),
//    the sheet crossed later on the right (V^dag, the path-ordered exponential of
//    Sec. 2, has later points on the left); with A_i = V d_i V^dag / (ig) the field
//    strength inside piece k is then sheet k's own, rotated by the completed pieces
//    (gauge covariance); sheets not reached yet (lambda_k = 0) are 1.
// 3. U_i = [V_A(x) V_A^dag(x+i)] [V_B(x) V_B^dag(x+i)] (i = x, y), U_z = 1 except the
//    periodic seam U_z(x_T, nz-1) = V_A(x_T, nz-1) V_B^dag(x_T, 0), at t0 and t0 - dt.
// 4. E_i(t0 - dt/2) = -i Log(U_i(t0) U_i^dag(t0 - dt)) / (a_i dt), principal Log.
// 5. rho = sum_i [E_i(x) - U_i^dag(x-i) E_i(x-i) U_i(x-i)] / a_i at U(t0); layers
//    z < nz/2 go to nucleus B, the others to nucleus A.
#include "internal.h"

namespace gl {

size_t ic_work_doubles(const Geom& g, int ng) { return (size_t)6 * 2 * ng * g.layer; }

__global__ void k_dft(const double* __restrict__ in, double* __restrict__ out, int nt, int nb, int mode,
                      double a_T, double m_ir, double uv_cut) {
  const int64_t n2 = (int64_t)nt * nt;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= nb * n2) return;
  const int b = (int)(tid / n2);
  const int y = (int)((tid / nt) % nt);
  const int x = (int)(tid % nt);
  const double* ib = in + (mode == 0 ? 1 : 2) * (int64_t)b * n2;
  double sr = 0.0, si = 0.0;
  if (mode == 0) {          // real in, forward along x: out[b][y][kx=x]
    for (int u = 0; u < nt; ++u) {
      double s, c;
      sincospi(2.0 * (double)((x * u) % nt) / nt, &s, &c);
      double v = ib[(int64_t)y * nt + u];
      sr += v * c; si -= v * s;
    }
  } else if (mode == 1 || mode == 2) {   // along y: out[b][ky=y][kx=x]
    const double sg = mode == 1 ? -1.0 : 1.0;
    for (int u = 0; u < nt; ++u) {
      double s, c;
      sincospi(2.0 * (double)((y * u) % nt) / nt, &s, &c);
      s *= sg;
      double vr = ib[2 * ((int64_t)u * nt + x)], vi = ib[2 * ((int64_t)u * nt + x) + 1];
      sr += vr * c - vi * s; si += vr * s + vi * c;
    }
    if (mode == 1) {
      double sy = sinpi((double)y / nt), sx = sinpi((double)x / nt);
      double k2 = (2.0 / a_T) * (2.0 / a_T) * (sy * sy + sx * sx);
      double f = 1.0 / (k2 + m_ir * m_ir);
      if (uv_cut > 0.0 && sqrt(k2) > uv_cut) f = 0.0;
      sr *= f; si *= f;
    }
  } else {                  // complex in, inverse along x, real out / nt^2
    for (int u = 0; u < nt; ++u) {
      double s, c;
      sincospi(2.0 * (double)((x * u) % nt) / nt, &s, &c);
      double vr = ib[2 * ((int64_t)y * nt + u)], vi = ib[2 * ((int64_t)y * nt + u) + 1];
      sr += vr * c - vi * s;
    }
    out[tid] = sr / (double)n2;
    return;
  }
  out[2 * tid] = sr;
  out[2 * tid + 1] = si;
}

template <typename Gd>
__device__ __forceinline__ typename Gd::Alg sheet_phi(const double* __restrict__ phi, int sheet, int nucleus,
                                                      int64_t t, int64_t layer) {
  typename Gd::Alg p;
  constexpr int NG = Gd::NG;
#pragma unroll
  for (int k = 0; k < NG; ++k) p.c[k] = phi[(((int64_t)sheet * 2 + nucleus) * NG + k) * layer + t];
  return p;
}
// V_N at transverse site t for cumulative profile weight lam of the whole nucleus
template <typename Gd>
__device__ typename Gd::Link wilson(const double* __restrict__ phi, int ns, int nucleus, int64_t t, int64_t layer,
                                    double lam) {
  typename Gd::Link V = Gd::expi(sheet_phi<Gd>(phi, 0, nucleus, t, layer), -fmin(fmax(ns * lam, 0.0), 1.0));
  for (int k = 1; k < ns; ++k) {
    const double lk = fmin(fmax(ns * lam - k, 0.0), 1.0);
    if (lk > 0.0) V = Gd::mul(V, Gd::expi(sheet_phi<Gd>(phi, k, nucleus, t, layer), -lk));
  }
  return V;
}

__device__ __forceinline__ double profileA(double z, double tau, const McvConst& mv) {
  return 0.5 * erfc(-(z - mv.zA + tau) / (1.4142135623730951 * mv.sigma));
}
__device__ __forceinline__ double profileB(double z, double tau, const McvConst& mv) {
  return 0.5 * erfc((z - mv.zB - tau) / (1.4142135623730951 * mv.sigma));
}

template <typename Gd>
__device__ typename Gd::Link ic_link(const double* __restrict__ phi, int ns, const Geom& g, int x, int y, int z,
                                     int i, double tau, double a_L, const McvConst& mv) {
  using L = typename Gd::Link;
  const int64_t t = (int64_t)y * g.nt + x;
  if (i == 2) {
    if (z != g.nz - 1) return Gd::one();
    L VA = wilson<Gd>(phi, ns, 0, t, g.layer, profileA((g.nz - 1) * a_L, tau, mv));
    L VB = wilson<Gd>(phi, ns, 1, t, g.layer, profileB(0.0, tau, mv));
    return Gd::mul_dag(VA, VB);
  }
  const int xp = i == 0 ? wrap_add(x, 1, g.nt) : x;
  const int yp = i == 1 ? wrap_add(y, 1, g.nt) : y;
  const int64_t tp = (int64_t)yp * g.nt + xp;
  const double zz = z * a_L;
  const double lA = profileA(zz, tau, mv), lB = profileB(zz, tau, mv);
  L UA = Gd::mul_dag(wilson<Gd>(phi, ns, 0, t, g.layer, lA), wilson<Gd>(phi, ns, 0, tp, g.layer, lA));
  L UB = Gd::mul_dag(wilson<Gd>(phi, ns, 1, t, g.layer, lB), wilson<Gd>(phi, ns, 1, tp, g.layer, lB));
  return Gd::mul(UA, UB);
}

// (launched with 256 threads: the bound lets the compiler use the registers of two waves per
// SIMD instead of spilling to fit 1024-thread blocks)
template <typename Gd, typename T>
__global__ void __launch_bounds__(256) k_ic_links(const double* __restrict__ phi, int ns, T* __restrict__ U, T* __restrict__ E, Geom g,
                           StepConst c, McvConst mv) {
  constexpr int NG = Gd::NG;
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  const int x = (int)(s % g.nt), y = (int)((s / g.nt) % g.nt), z = (int)(s / g.layer);
  for (int i = 0; i < 3; ++i) {
    typename Gd::Link U0 = ic_link<Gd>(phi, ns, g, x, y, z, i, 0.0, c.a[2], mv);
    typename Gd::Link U1 = ic_link<Gd>(phi, ns, g, x, y, z, i, -c.dt, c.a[2], mv);
    typename Gd::Alg e = Gd::logi(Gd::mul_dag(U0, U1));
    const double k = 1.0 / (c.a[i] * c.dt);
    for (int q = 0; q < NG; ++q) e.c[q] *= k;
    store_link(U0, U, i, (uint32_t)s, g.Vp);
    store_alg(e, E, i, (uint32_t)s, g.Vp);
  }
}

template <typename Gd, typename T>
__global__ void k_ic_gauss(const T* __restrict__ U, const T* __restrict__ E, const T* __restrict__ F2,
                           double scale, T* __restrict__ rhoA, T* __restrict__ rhoB, Geom g, StepConst c) {
  constexpr int NG = Gd::NG;
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  const int64_t Vp = g.Vp;
  Site x;
  x.x = (int)(s % g.nt); x.y = (int)((s / g.nt) % g.nt); x.z = (int)(s / g.layer);
  typename Gd::Alg r = Gd::alg_zero();
  for (int i = 0; i < 3; ++i) {
    const int64_t sm = idx(g, shifted(g, x, i, -1));
    typename Gd::Link Um;
    load_link(Um, U, i, sm, Vp);
    typename Gd::Alg eh, em;
    load_alg(eh, E, i, s, Vp);
    load_alg(em, E, i, sm, Vp);
    if (F2) {
      typename Gd::Alg fh, fm;
      load_alg(fh, F2, i, s, Vp);
      load_alg(fm, F2, i, sm, Vp);
      for (int q = 0; q < NG; ++q) { eh.c[q] += scale * fh.c[q]; em.c[q] += scale * fm.c[q]; }
    }
    typename Gd::Alg tr = Gd::transport(Um, em);
    for (int q = 0; q < NG; ++q) r.c[q] += (eh.c[q] - tr.c[q]) / c.a[i];
  }
  typename Gd::Alg zero = Gd::alg_zero();
  const bool isB = x.z < g.nz / 2;
  store_alg(isB ? r : zero, rhoB, 0, s, Vp);
  store_alg(isB ? zero : r, rhoA, 0, s, Vp);
}

void launch_ic_phi(double* work, double* phi_out, int ng, const Geom& g, const StepConst& c, const McvConst& mv,
                   hipStream_t st) {
  const int nb = 2 * ng;
  const int64_t m = (int64_t)nb * g.layer;
  double* c1 = work + 2 * m;
  double* c2 = work + 4 * m;
  const int bs = 256;
  const unsigned gb = (unsigned)((m + bs - 1) / bs);
  hipLaunchKernelGGL(k_dft, dim3(gb), dim3(bs), 0, st, work, c1, g.nt, nb, 0, c.a[0], mv.m_ir, mv.uv_cut);
  hipLaunchKernelGGL(k_dft, dim3(gb), dim3(bs), 0, st, c1, c2, g.nt, nb, 1, c.a[0], mv.m_ir, mv.uv_cut);
  hipLaunchKernelGGL(k_dft, dim3(gb), dim3(bs), 0, st, c2, c1, g.nt, nb, 2, c.a[0], mv.m_ir, mv.uv_cut);
  hipLaunchKernelGGL(k_dft, dim3(gb), dim3(bs), 0, st, c1, phi_out, g.nt, nb, 3, c.a[0], mv.m_ir, mv.uv_cut);
}

template <typename G, typename T>
void launch_ic_fields(const double* phi, int ns, T* U, T* E, T* rhoA, T* rhoB, const Geom& g, const StepConst& c,
                      const McvConst& mv, hipStream_t st) {
  using Gd = typename GroupOf<G::NC, double>::type;
  const int bs = 256;
  const unsigned sb = (unsigned)((g.V + bs - 1) / bs);
  hipLaunchKernelGGL((k_ic_links<Gd, T>), dim3(sb), dim3(bs), 0, st, phi, ns, U, E, g, c, mv);
  // the semi-implicit scheme conserves D.(E + dt f1(U(t0), U(t0 - dt))) - rho instead;
  // its caller builds f1 and sets the charges through launch_gauss_charges
  if (c.scheme == 1) return;
  hipLaunchKernelGGL((k_ic_gauss<Gd, T>), dim3(sb), dim3(bs), 0, st, U, E, (const T*)nullptr, 0.0, rhoA, rhoB, g, c);
}

template <typename G, typename T>
void launch_gauss_charges(const T* U, const T* E, const T* F2, double scale, T* rhoA, T* rhoB, const Geom& g,
                          const StepConst& c, hipStream_t st) {
  using Gd = typename GroupOf<G::NC, double>::type;
  const int bs = 256;
  const unsigned sb = (unsigned)((g.V + bs - 1) / bs);
  hipLaunchKernelGGL((k_ic_gauss<Gd, T>), dim3(sb), dim3(bs), 0, st, U, E, F2, scale, rhoA, rhoB, g, c);
}

#define GL_GC_INST(G, T) \
  template void launch_gauss_charges<G, T>(const T*, const T*, const T*, double, T*, T*, const Geom&, const StepConst&, hipStream_t);
GL_GC_INST(Su2<double>, double)
GL_GC_INST(Su3<double>, double)
GL_GC_INST(Su2<float>, float)
GL_GC_INST(Su3<float>, float)
#define GL_IC_INST(G, T) \
  template void launch_ic_fields<G, T>(const double*, int, T*, T*, T*, T*, const Geom&, const StepConst&, \
                                       const McvConst&, hipStream_t);
GL_IC_INST(Su2<double>, double)
GL_IC_INST(Su3<double>, double)
GL_IC_INST(Su2<float>, float)
GL_IC_INST(Su3<float>, float)

}  // namespace gl
