// Reverse mode of the leapfrog step with the CPIC hop (Sec. 3: eqs. lattice_1, lattice_2,
// plaquette, continuity and the transport rule of the hop), for gradients of a loss of the
// final state with respect to the initial electric field and charges.
//
// Cotangents (double precision, plain structure of arrays [dir][a][V]):
//   lam_i(x)  = dL/d eps^a for the left variation U_i(x) -> exp(i eps^a t^a) U_i(x)
//   ebar_i(x) = dL/dE_i^a(x),  rbarA(x), rbarB(x) = dL/drho^a(x) at lab positions.
// Hermitian matrices H enter products in the form i H (SU(2): a pure quaternion, SU(3):
// an anti-hermitian matrix); P(.) of such a product returns its hermitian components.
//
// The step  rho' = hop(rho, U);  E' = E + dt (F(U) + j);  U'_i = exp(i c_i E'_i) U_i
// (c_i = a_i dt) is reversed in three kernels:
//  ra: lam_i <- W^dag lam'_i W,  ebar_i <- ebar'_i + c_i int_0^1 W_s^dag lam'_i W_s ds
//      (W = exp(i c_i E'_i), W_s = exp(i s c_i E'_i)); ebar then holds dL/dE' = dL/dE.
//  r1: per plaquette square (corner x, plane (i,j)) the four force terms that contain it,
//      F_i(x), F_j(x), F_i(x+j), F_j(x+i), with cotangents Fbar = dt ebar, fold into one
//      hermitian Omega in the frame of W = U_{i,j}(x):
//        Omega = c_ij [Fbar_i(x) - U_j(x) Fbar_i(x+j) U_j^dag(x)]
//              - c_ji [Fbar_j(x) - U_i(x) Fbar_j(x+i) U_i^dag(x)],   c_ij = -1/(a_i a_j^2),
//      and K = P(W i Omega), K' = P(i Omega W) are stored; the two corner links inside the
//      transports get the extra commutator terms described at k_adj_r1.
//  r2: each link gathers its four squares: for U_k(y) and m != k, with (i,j) the sorted
//      plane, +K(y) - U_m^dag K'(y-m) U_m (k = i) or +U_m^dag K(y-m) U_m - K'(y) (k = j),
//      U_m = U_m(y-m); on hop steps the charge transport adds to lam_z and moves the charge
//      cotangents back one cell.
#include "internal.h"
#include "stencil.h"
#include "adjoint.h"

namespace gl {

// ---- plain [dir][a][V] double arrays -------------------------------------------
template <typename A> GL_HD void ld(A& a, const double* __restrict__ f, int dir, int64_t V, uint32_t s) {
  constexpr int NG = sizeof(a.c) / sizeof(a.c[0]);
  const double* p = f + (int64_t)dir * NG * V + s;
#pragma unroll
  for (int k = 0; k < NG; ++k) a.c[k] = p[k * V];
}
template <typename A> GL_HD void st(const A& a, double* __restrict__ f, int dir, int64_t V, uint32_t s) {
  constexpr int NG = sizeof(a.c) / sizeof(a.c[0]);
  double* p = f + (int64_t)dir * NG * V + s;
#pragma unroll
  for (int k = 0; k < NG; ++k) p[k * V] = a.c[k];
}

GL_HD bool site_of(const Geom& g, uint32_t b, uint32_t nb, uint32_t t, uint32_t bs, Site& x, uint32_t& s) {
  s = xcd_remap(b, nb) * bs + t;
  if (s >= (uint32_t)g.V) return false;
  x.x = (int)(s % (uint32_t)g.nt);
  x.y = (int)((s / (uint32_t)g.nt) % (uint32_t)g.nt);
  x.z = (int)(s / (uint32_t)g.layer);
  return true;
}

// Block sum of one double per thread into out[blockIdx.x] (256 threads).
__device__ __forceinline__ void block_sum(double v, double* __restrict__ out) {
  __shared__ double red[256];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// ---- loss and its seed -----------------------------------------------------------
// L = a_x a_y a_z sum_{z0 <= z < z1} [ 1/2 sum_i |E_i|^2 + sum_{i<j} 2/(a_i a_j)^2 Re Tr(1 - U_{i,j}) ]
// and, when SEED, lam = scale dL/dU (left), ebar = scale dL/dE, rbar = 0.  For link U_k(y)
// the squares of L that contain it are U_{k,m}(y) (corner y) and U_{k,-m}(y) (corner y - m);
// d Re Tr(P)/d eps = -P(P)/2 for the loop P that starts with the link.
template <typename Gd, typename S, bool SEED>
__global__ void __launch_bounds__(256) k_adj_loss(const S* __restrict__ U, const S* __restrict__ E, Geom g,
                                                  double ax, double ay, double az, int z0, int z1, double scale,
                                                  double* __restrict__ lam, double* __restrict__ ebar,
                                                  double* __restrict__ rA, double* __restrict__ rB,
                                                  double* __restrict__ partial) {
  using L = typename Gd::Link;
  using A = typename Gd::Alg;
  constexpr int NG = Gd::NG;
  const double a[3] = {ax, ay, az};
  const double a3 = ax * ay * az;
  Site y;
  uint32_t s;
  double contrib = 0.0;
  if (site_of(g, blockIdx.x, gridDim.x, threadIdx.x, blockDim.x, y, s)) {
    const bool in = y.z >= z0 && y.z < z1;
    const int zm = y.z == 0 ? g.nz - 1 : y.z - 1;
    const bool in_m = zm >= z0 && zm < z1;   // corner y - z
    double e2 = 0.0;
    for (int i = 0; i < 3; ++i) {
      A e;
      load_alg(e, E, i, s, g.Vp);
      for (int k = 0; k < NG; ++k) e2 += e.c[k] * e.c[k];
      if (SEED) {
        for (int k = 0; k < NG; ++k) e.c[k] = in ? scale * a3 * e.c[k] : 0.0;
        st(e, ebar, i, g.V, s);
      }
    }
    double b = 0.0;
    for (int k = 0; k < 3; ++k) {
      L Uk;
      load_link(Uk, U, k, s, g.Vp);
      A acc = Gd::alg_zero();
      const Site ypk = shifted(g, y, k, +1);
      for (int m = 0; m < 3; ++m) {
        if (m == k) continue;
        const double w = a3 / (a[k] * a[k] * a[m] * a[m]);
        L Am, Bk, Cm;
        // U_{k,m}(y) = U_k(y) U_m(y+k) U_k^dag(y+m) U_m^dag(y)
        load_link(Am, U, m, idx(g, ypk), g.Vp);
        load_link(Bk, U, k, idx(g, shifted(g, y, m, +1)), g.Vp);
        load_link(Cm, U, m, s, g.Vp);
        const L P = Gd::mul_dag(Gd::mul_dag(Gd::mul(Uk, Am), Bk), Cm);
        if (k < m) b += 2.0 / (a[k] * a[k] * a[m] * a[m]) * ((double)Gd::NC - Gd::retr(P));
        const bool in_m_dir = m == 2 ? in_m : in;
        if (SEED) {
          if (in) axpy(acc, w, Gd::proj(P));
          if (in_m_dir) {
            // U_{k,-m}(y) = U_k(y) U_m^dag(y+k-m) U_k^dag(y-m) U_m(y-m)
            const Site ymm = shifted(g, y, m, -1);
            load_link(Am, U, m, idx(g, shifted(g, ypk, m, -1)), g.Vp);
            load_link(Bk, U, k, idx(g, ymm), g.Vp);
            load_link(Cm, U, m, idx(g, ymm), g.Vp);
            const L Pn = Gd::mul(Gd::mul_dag(Gd::mul_dag(Uk, Am), Bk), Cm);
            axpy(acc, w, Gd::proj(Pn));
          }
        }
      }
      if (SEED) {
        for (int q = 0; q < NG; ++q) acc.c[q] *= scale;
        st(acc, lam, k, g.V, s);
      }
    }
    if (SEED) {
      const A z = Gd::alg_zero();
      st(z, rA, 0, g.V, s);
      st(z, rB, 0, g.V, s);
    }
    contrib = in ? a3 * (0.5 * e2 + b) : 0.0;
  }
  block_sum(contrib, partial);
}

__global__ void __launch_bounds__(256) k_sum(const double* __restrict__ partial, int n, double* __restrict__ out) {
  double v = 0.0;
  for (int k = threadIdx.x; k < n; k += blockDim.x) v += partial[k];
  block_sum(v, out);
}

// ---- ra: reverse of the link update -----------------------------------------------
template <typename Gd, typename S>
__global__ void __launch_bounds__(256) k_adj_ra(const S* __restrict__ E1, Geom g, double ax, double ay, double az,
                                                double dt, double* __restrict__ lam, double* __restrict__ ebar) {
  using L = typename Gd::Link;
  using A = typename Gd::Alg;
  Site x;
  uint32_t s;
  if (!site_of(g, blockIdx.x, gridDim.x, threadIdx.x, blockDim.x, x, s)) return;
  const int i = blockIdx.y;
  const double c = (i == 0 ? ax : i == 1 ? ay : az) * dt;
  A e, lp, ep;
  load_alg(e, E1, i, s, g.Vp);
  ld(lp, lam, i, g.V, s);
  ld(ep, ebar, i, g.V, s);
  const L W = Gd::expi(e, c);
  const A l = Gd::transport(W, lp);
  axpy(ep, 1.0, dexp_transpose<Gd>(e, c, lp));
  st(l, lam, i, g.V, s);
  st(ep, ebar, i, g.V, s);
}

// ---- r1: one hermitian cotangent per plaquette square -------------------------------
// One thread per site x, the three planes in turn.  Besides K, K' it adds to lam_i(x) and
// lam_j(x) the derivative of the transports U_j(x) . U_j^dag(x) and U_i(x) . U_i^dag(x)
// that rotate the terms of F_i(x+j) and F_j(x+i) into the frame of W:
//   lam_i(x) += P([i T4, W]),  lam_j(x) -= P([i T3, W]),
//   T3 = dt c_ij U_j(x) ebar_i(x+j) U_j^dag(x),  T4 = dt c_ji U_i(x) ebar_j(x+i) U_i^dag(x).
template <typename Gd, typename S>
__global__ void __launch_bounds__(256) k_adj_r1(const S* __restrict__ U, Geom g, double ax, double ay, double az,
                                                double dt, const double* __restrict__ ebar, double* __restrict__ K,
                                                double* __restrict__ lam) {
  using L = typename Gd::Link;
  using A = typename Gd::Alg;
  constexpr int NG = Gd::NG;
  Site x;
  uint32_t s;
  if (!site_of(g, blockIdx.x, gridDim.x, threadIdx.x, blockDim.x, x, s)) return;
  const double a[3] = {ax, ay, az};
#pragma unroll 1
  for (int p = 0; p < 3; ++p) {              // plane (0,1), (0,2), (1,2)
    const int i = p == 2 ? 1 : 0, j = p == 0 ? 1 : 2;
    const double cij = -dt / (a[i] * a[j] * a[j]), cji = -dt / (a[j] * a[i] * a[i]);
    const Site xpi = shifted(g, x, i, +1), xpj = shifted(g, x, j, +1);
    L Ui, Uj, Ujpi, Uipj;
    load_link(Ui, U, i, s, g.Vp);
    load_link(Uj, U, j, s, g.Vp);
    load_link(Ujpi, U, j, idx(g, xpi), g.Vp);
    load_link(Uipj, U, i, idx(g, xpj), g.Vp);
    A ei, ej, t3, t4;
    ld(ei, ebar, i, g.V, s);
    ld(ej, ebar, j, g.V, s);
    ld(t3, ebar, i, g.V, idx(g, xpj));
    t3 = Gd::transport_inv(Uj, t3);
    ld(t4, ebar, j, g.V, idx(g, xpi));
    t4 = Gd::transport_inv(Ui, t4);
    A om;
    for (int k = 0; k < NG; ++k) {
      t3.c[k] *= cij;
      t4.c[k] *= cji;
      om.c[k] = cij * ei.c[k] - cji * ej.c[k] - t3.c[k] + t4.c[k];
    }
    const L W = Gd::mul_dag(Gd::mul_dag(Gd::mul(Ui, Ujpi), Uipj), Uj);
    const L Oh = AdjOps<Gd>::anti(om);
    st(Gd::proj(Gd::mul(W, Oh)), K, 2 * p, g.V, s);
    st(Gd::proj(Gd::mul(Oh, W)), K, 2 * p + 1, g.V, s);
    A l;
    ld(l, lam, i, g.V, s);
    axpy(l, 1.0, Gd::proj(commut<Gd>(AdjOps<Gd>::anti(t4), W)));
    st(l, lam, i, g.V, s);
    ld(l, lam, j, g.V, s);
    axpy(l, -1.0, Gd::proj(commut<Gd>(AdjOps<Gd>::anti(t3), W)));
    st(l, lam, j, g.V, s);
  }
}

// ---- r2: gather of the link cotangents; hop reverse ---------------------------------
// Charges: rho_A at state s+1 in co-moving slots with offset offA1, rho_B at state s with
// offset offB0.
template <typename Gd, typename S, bool HOP>
__global__ void __launch_bounds__(256) k_adj_r2(const S* __restrict__ U, const S* __restrict__ rhoA1,
                                                const S* __restrict__ rhoB0, int offA1, int offB0, Geom g, double aL,
                                                const double* __restrict__ ebar, const double* __restrict__ K,
                                                double* __restrict__ lam, const double* __restrict__ rAin,
                                                const double* __restrict__ rBin, double* __restrict__ rAout,
                                                double* __restrict__ rBout) {
  using L = typename Gd::Link;
  using A = typename Gd::Alg;
  constexpr int NG = Gd::NG;
  Site y;
  uint32_t s;
  if (!site_of(g, blockIdx.x, gridDim.x, threadIdx.x, blockDim.x, y, s)) return;
  for (int k = 0; k < 3; ++k) {
    A acc, t;
    ld(acc, lam, k, g.V, s);
    for (int m = 0; m < 3; ++m) {
      if (m == k) continue;
      const int p = k + m - 1;
      const uint32_t sm = idx(g, shifted(g, y, m, -1));
      L Um;
      load_link(Um, U, m, sm, g.Vp);
      if (k < m) {
        ld(t, K, 2 * p, g.V, s);
        axpy(acc, 1.0, t);
        ld(t, K, 2 * p + 1, g.V, sm);
        axpy(acc, -1.0, Gd::transport(Um, t));
      } else {
        ld(t, K, 2 * p, g.V, sm);
        axpy(acc, 1.0, Gd::transport(Um, t));
        ld(t, K, 2 * p + 1, g.V, s);
        axpy(acc, -1.0, t);
      }
    }
    if (HOP && k == 2) {
      L Uz;
      load_link(Uz, U, 2, s, g.Vp);
      A abar, ez, ra1, rb0, bin;
      ld(abar, rAin, 0, g.V, s);
      ld(ez, ebar, 2, g.V, s);
      axpy(abar, aL, ez);                                   // dL/drho_A'(y)
      load_alg(ra1, rhoA1, 0, site_index(g, y.x, y.y, slotA(y.z, offA1, g.nz)), g.Vp);
      load_alg(rb0, rhoB0, 0, site_index(g, y.x, y.y, slotB(y.z, offB0, g.nz)), g.Vp);
      ld(bin, rBin, 0, g.V, idx(g, shifted(g, y, 2, +1)));
      A R = Gd::transport_inv(Uz, bin);                     // U_z(y) rbarB'(y+z) U_z^dag(y)
      axpy(acc, 1.0, Gd::proj(commut<Gd>(AdjOps<Gd>::anti(ra1), AdjOps<Gd>::anti(abar))));
      axpy(acc, 1.0, Gd::proj(commut<Gd>(AdjOps<Gd>::anti(R), AdjOps<Gd>::anti(rb0))));
      axpy(R, -aL, ez);
      st(R, rBout, 0, g.V, s);
    }
    st(acc, lam, k, g.V, s);
  }
  if (HOP) {
    // rbarA(y) = U_z^dag(y-z) [rbarA'(y-z) + a_L ebar_z(y-z)] U_z(y-z)
    const uint32_t sm = idx(g, shifted(g, y, 2, -1));
    L Uz;
    load_link(Uz, U, 2, sm, g.Vp);
    A abar, ez;
    ld(abar, rAin, 0, g.V, sm);
    ld(ez, ebar, 2, g.V, sm);
    axpy(abar, aL, ez);
    st(Gd::transport(Uz, abar), rAout, 0, g.V, s);
  }
  (void)NG;
}

// ---- device state transfer (plain double arrays <-> tiled storage) --------------------
// Algebra fields (width n_g): src/dst [dir][comp][V] double; charges at physical layer z
// live in their co-moving slot.
template <typename S, int W>
__global__ void __launch_bounds__(256) k_pack(const double* __restrict__ src, const double* __restrict__ amp,
                                              S* __restrict__ dst, Geom g, int ndir) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= (uint32_t)g.V) return;
  const int d = blockIdx.y;
  const double f = amp ? amp[s] : 1.0;
  double v[W];
  for (int k = 0; k < W; ++k) v[k] = f * src[((int64_t)d * W + k) * g.V + s];
  store_comps<double, S, W>(v, field_dir(dst, d, W, g.Vp), s);
  (void)ndir;
}
template <typename S, int W>
__global__ void __launch_bounds__(256) k_unpack(const S* __restrict__ src, double* __restrict__ dst, Geom g, int off,
                                                int kind) {
  // kind 0: plain field; 1: co-moving nucleus A; 2: co-moving nucleus B
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= (uint32_t)g.V) return;
  const int d = blockIdx.y;
  const int x = (int)(s % (uint32_t)g.nt), y = (int)((s / (uint32_t)g.nt) % (uint32_t)g.nt);
  const int z = (int)(s / (uint32_t)g.layer);
  const int zs = kind == 1 ? slotA(z, off, g.nz) : kind == 2 ? slotB(z, off, g.nz) : z;
  double v[W];
  load_comps<double, S, W>(v, field_dir(src, d, W, g.Vp), site_index(g, x, y, zs));
  for (int k = 0; k < W; ++k) dst[((int64_t)d * W + k) * g.V + s] = v[k];
}

// Links: plain [dir][host reals][V] double <-> the storage of load_link / store_link.
template <typename Gs, typename S>
__global__ void __launch_bounds__(256) k_pack_links(const double* __restrict__ src, S* __restrict__ dst, Geom g) {
  using L = typename Gs::Link;
  constexpr int R = Gs::R;
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= (uint32_t)g.V) return;
  const int d = blockIdx.y;
  double v[R];
  for (int k = 0; k < R; ++k) v[k] = src[((int64_t)d * R + k) * g.V + s];
  L l;
  if constexpr (R == 4) {
    for (int k = 0; k < 4; ++k) l.q[k] = v[k];
  } else {
    for (int r = 0; r < 3; ++r)
      for (int k = 0; k < 3; ++k) { l.re[r][k] = v[2 * (3 * r + k)]; l.im[r][k] = v[2 * (3 * r + k) + 1]; }
  }
  store_link(l, dst, d, s, g.Vp);
}
template <typename Gs, typename S>
__global__ void __launch_bounds__(256) k_unpack_links(const S* __restrict__ src, double* __restrict__ dst, Geom g) {
  using L = typename Gs::Link;
  constexpr int R = Gs::R;
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= (uint32_t)g.V) return;
  const int d = blockIdx.y;
  L l;
  load_link(l, src, d, s, g.Vp);
  double v[R];
  if constexpr (R == 4) {
    for (int k = 0; k < 4; ++k) v[k] = l.q[k];
  } else {
    for (int r = 0; r < 3; ++r)
      for (int k = 0; k < 3; ++k) { v[2 * (3 * r + k)] = l.re[r][k]; v[2 * (3 * r + k) + 1] = l.im[r][k]; }
  }
  for (int k = 0; k < R; ++k) dst[((int64_t)d * R + k) * g.V + s] = v[k];
}

// dL/d alpha(x) = sum_a base^a(x) rbar^a(x) (per-cell amplitude of the charges); base in the
// plain layout, or (base == null) the tiled charges at offset off of nucleus `which`.
template <typename Gd, typename S>
__global__ void __launch_bounds__(256) k_amp(const double* __restrict__ rbar, const double* __restrict__ base,
                                             const S* __restrict__ rho, int off, int which, Geom g,
                                             double* __restrict__ out) {
  using A = typename Gd::Alg;
  constexpr int NG = Gd::NG;
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= (uint32_t)g.V) return;
  A r, b;
  ld(r, rbar, 0, g.V, s);
  if (base) {
    ld(b, base, 0, g.V, s);
  } else {
    const int x = (int)(s % (uint32_t)g.nt), y = (int)((s / (uint32_t)g.nt) % (uint32_t)g.nt);
    const int z = (int)(s / (uint32_t)g.layer);
    const int zs = which == 0 ? slotA(z, off, g.nz) : slotB(z, off, g.nz);
    load_alg(b, rho, 0, site_index(g, x, y, zs), g.Vp);
  }
  double v = 0.0;
  for (int k = 0; k < NG; ++k) v += r.c[k] * b.c[k];
  out[s] = v;
}

// ---- launchers ---------------------------------------------------------------------
static inline unsigned nblocks(const Geom& g) { return (unsigned)((g.V + 255) / 256); }

template <typename G, typename S>
void launch_adj_loss(const S* U, const S* E, const Geom& g, const double* a, int z0, int z1, double scale,
                     double* lam, double* ebar, double* rA, double* rB, double* partial, double* out,
                     hipStream_t stm) {
  using Gd = typename GroupOf<G::NC, double>::type;
  const unsigned nb = nblocks(g);
  if (lam)
    hipLaunchKernelGGL((k_adj_loss<Gd, S, true>), dim3(nb), dim3(256), 0, stm, U, E, g, a[0], a[1], a[2], z0, z1,
                       scale, lam, ebar, rA, rB, partial);
  else
    hipLaunchKernelGGL((k_adj_loss<Gd, S, false>), dim3(nb), dim3(256), 0, stm, U, E, g, a[0], a[1], a[2], z0, z1,
                       scale, lam, ebar, rA, rB, partial);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, stm, partial, (int)nb, out);
}
size_t adj_loss_partials(const Geom& g) { return nblocks(g); }

template <typename G, typename S>
void launch_adj_step(const S* U0, const S* E1, const S* rhoA1, const S* rhoB0, int offA1, int offB0, bool hop,
                     const Geom& g, const double* a, double dt, double* lam, double* ebar, double* K,
                     const double* rAin, const double* rBin, double* rAout, double* rBout, hipStream_t stm) {
  using Gd = typename GroupOf<G::NC, double>::type;
  const unsigned nb = nblocks(g);
  hipLaunchKernelGGL((k_adj_ra<Gd, S>), dim3(nb, 3), dim3(256), 0, stm, E1, g, a[0], a[1], a[2], dt, lam, ebar);
  hipLaunchKernelGGL((k_adj_r1<Gd, S>), dim3(nb), dim3(256), 0, stm, U0, g, a[0], a[1], a[2], dt, ebar, K, lam);
  if (hop)
    hipLaunchKernelGGL((k_adj_r2<Gd, S, true>), dim3(nb), dim3(256), 0, stm, U0, rhoA1, rhoB0, offA1, offB0, g, a[2],
                       ebar, K, lam, rAin, rBin, rAout, rBout);
  else
    hipLaunchKernelGGL((k_adj_r2<Gd, S, false>), dim3(nb), dim3(256), 0, stm, U0, rhoA1, rhoB0, offA1, offB0, g,
                       a[2], ebar, K, lam, rAin, rBin, rAout, rBout);
}

template <typename G, typename S>
void launch_pack(const double* src, const double* amp, S* dst, const Geom& g, int ndir, int width, hipStream_t stm) {
  const dim3 grid(nblocks(g), (unsigned)ndir);
  if (width == 3) hipLaunchKernelGGL((k_pack<S, 3>), grid, dim3(256), 0, stm, src, amp, dst, g, ndir);
  else hipLaunchKernelGGL((k_pack<S, 8>), grid, dim3(256), 0, stm, src, amp, dst, g, ndir);
}
template <typename G, typename S>
void launch_unpack(const S* src, double* dst, const Geom& g, int ndir, int width, int off, int kind, hipStream_t stm) {
  const dim3 grid(nblocks(g), (unsigned)ndir);
  if (width == 3) hipLaunchKernelGGL((k_unpack<S, 3>), grid, dim3(256), 0, stm, src, dst, g, off, kind);
  else hipLaunchKernelGGL((k_unpack<S, 8>), grid, dim3(256), 0, stm, src, dst, g, off, kind);
}
template <typename G, typename S>
void launch_pack_links(const double* src, S* dst, const Geom& g, hipStream_t stm) {
  using Gd = typename GroupOf<G::NC, double>::type;
  hipLaunchKernelGGL((k_pack_links<Gd, S>), dim3(nblocks(g), 3), dim3(256), 0, stm, src, dst, g);
}
template <typename G, typename S>
void launch_unpack_links(const S* src, double* dst, const Geom& g, hipStream_t stm) {
  using Gd = typename GroupOf<G::NC, double>::type;
  hipLaunchKernelGGL((k_unpack_links<Gd, S>), dim3(nblocks(g), 3), dim3(256), 0, stm, src, dst, g);
}
template <typename G, typename S>
void launch_amp(const double* rbar, const double* base, const S* rho, int off, int which, const Geom& g, double* out,
                hipStream_t stm) {
  using Gd = typename GroupOf<G::NC, double>::type;
  hipLaunchKernelGGL((k_amp<Gd, S>), dim3(nblocks(g)), dim3(256), 0, stm, rbar, base, rho, off, which, g, out);
}

#define GL_ADJ_INST(G, S)                                                                                          \
  template void launch_adj_loss<G, S>(const S*, const S*, const Geom&, const double*, int, int, double, double*,  \
                                      double*, double*, double*, double*, double*, hipStream_t);                  \
  template void launch_adj_step<G, S>(const S*, const S*, const S*, const S*, int, int, bool, const Geom&,        \
                                      const double*, double, double*, double*, double*, const double*,            \
                                      const double*, double*, double*, hipStream_t);                              \
  template void launch_pack<G, S>(const double*, const double*, S*, const Geom&, int, int, hipStream_t);          \
  template void launch_unpack<G, S>(const S*, double*, const Geom&, int, int, int, int, hipStream_t);             \
  template void launch_pack_links<G, S>(const double*, S*, const Geom&, hipStream_t);                             \
  template void launch_unpack_links<G, S>(const S*, double*, const Geom&, hipStream_t);                           \
  template void launch_amp<G, S>(const double*, const double*, const S*, int, int, const Geom&, double*,          \
                                 hipStream_t);
GL_ADJ_INST(Su2<double>, double)
GL_ADJ_INST(Su3<double>, double)
GL_ADJ_INST(Su2<float>, float)
GL_ADJ_INST(Su3<float>, float)

}  // namespace gl
