// SU(2) / SU(3) algebra for the lattice kernels (host + device, templated on the
// real type T = double or float).
//
// Conventions (Sec. 2: the generators t^a are hermitian and traceless):
//   t^a = sigma^a/2 (SU(2)) or lambda^a/2 (SU(3)), Tr t^a t^b = delta^ab/2.
//   A Lie-algebra element is stored by its real components X^a = 2 Tr(t^a X).
//   SU(2) links are unit quaternions U = q0 + i (q1 s1 + q2 s2 + q3 s3); the real
//   linear span of such matrices is closed under +, * and ^dag, so staple sums use
//   the same 4-real type.  SU(3) links are full 3x3 complex matrices (18 reals).
//   proj(M) returns the components of the hermitian traceless part of
//   (M - M^dag)/(2i); the paper's [M]_ah (Sec. 3, eq. lattice_1) is i proj(M).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#define GL_HD __host__ __device__ __forceinline__

namespace gl {

template <typename T> struct Alg2 { T c[3]; };
template <typename T> struct Alg3 { T c[8]; };

template <typename T> struct Q2 { T q[4]; };                 // SU(2) span element
template <typename T> struct M3 { T re[3][3]; T im[3][3]; };  // 3x3 complex

template <typename T> GL_HD T sqr(T x) { return x * x; }
// a * b + c with one rounding (v_fma_f64 / v_fma_f32); products below are written as
// chains of these so that every term costs one instruction
GL_HD double fmx(double a, double b, double c) { return __builtin_fma(a, b, c); }
GL_HD float fmx(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <typename T> GL_HD void sincos_r(T x, T* s, T* c);
template <> GL_HD void sincos_r<double>(double x, double* s, double* c) { sincos(x, s, c); }
template <> GL_HD void sincos_r<float>(float x, float* s, float* c) { sincosf(x, s, c); }

// ----------------------------------------------------------------------------
// SU(2)
// ----------------------------------------------------------------------------
template <typename T> struct Su2 {
  static constexpr int NC = 2, NG = 3, R = 4;
  using Real = T;
  using Link = Q2<T>;
  using Alg = Alg2<T>;

  static GL_HD Link zero() { Link r; for (int k = 0; k < 4; ++k) r.q[k] = T(0); return r; }
  static GL_HD Link one() { Link r = zero(); r.q[0] = T(1); return r; }
  static GL_HD Alg alg_zero() { Alg r; for (int k = 0; k < 3; ++k) r.c[k] = T(0); return r; }

  // (a0 + i a.s)(b0 + i b.s) = a0 b0 - a.b + i (a0 b + b0 a - a x b).s
  static GL_HD Link mul(const Link& a, const Link& b) {
    Link r;
    r.q[0] = a.q[0] * b.q[0] - a.q[1] * b.q[1] - a.q[2] * b.q[2] - a.q[3] * b.q[3];
    r.q[1] = a.q[0] * b.q[1] + b.q[0] * a.q[1] - (a.q[2] * b.q[3] - a.q[3] * b.q[2]);
    r.q[2] = a.q[0] * b.q[2] + b.q[0] * a.q[2] - (a.q[3] * b.q[1] - a.q[1] * b.q[3]);
    r.q[3] = a.q[0] * b.q[3] + b.q[0] * a.q[3] - (a.q[1] * b.q[2] - a.q[2] * b.q[1]);
    return r;
  }
  static GL_HD Link dag(const Link& a) { Link r; r.q[0] = a.q[0]; r.q[1] = -a.q[1]; r.q[2] = -a.q[2]; r.q[3] = -a.q[3]; return r; }
  static GL_HD Link mul_dag(const Link& a, const Link& b) { return mul(a, dag(b)); }   // a b^dag
  static GL_HD Link dag_mul(const Link& a, const Link& b) { return mul(dag(a), b); }   // a^dag b
  static GL_HD void add_to(Link& acc, const Link& a, T s) { for (int k = 0; k < 4; ++k) acc.q[k] += s * a.q[k]; }
  static GL_HD void acc_mul_dag(Link& r, const Link& a, const Link& b) { add_to(r, mul_dag(a, b), T(1)); }
  static GL_HD void acc_dag_mul(Link& r, const Link& a, const Link& b) { add_to(r, dag_mul(a, b), T(1)); }
  static GL_HD void scale(Link& r, T s) { for (int k = 0; k < 4; ++k) r.q[k] *= s; }
  // (U - U^dag)/(2i) = q.s  ->  components 2 q_a
  static GL_HD Alg proj(const Link& m) { Alg r; r.c[0] = 2 * m.q[1]; r.c[1] = 2 * m.q[2]; r.c[2] = 2 * m.q[3]; return r; }
  static GL_HD T retr(const Link& m) { return 2 * m.q[0]; }               // Re Tr
  // Re Tr(a b^dag)
  static GL_HD T retr_mul_dag(const Link& a, const Link& b) {
    return 2 * (a.q[0] * b.q[0] + a.q[1] * b.q[1] + a.q[2] * b.q[2] + a.q[3] * b.q[3]);
  }
  // proj(a b): only the vector part of the product
  static GL_HD Alg proj_mul(const Link& a, const Link& b) {
    Alg r;
    r.c[0] = 2 * (a.q[0] * b.q[1] + b.q[0] * a.q[1] - (a.q[2] * b.q[3] - a.q[3] * b.q[2]));
    r.c[1] = 2 * (a.q[0] * b.q[2] + b.q[0] * a.q[2] - (a.q[3] * b.q[1] - a.q[1] * b.q[3]));
    r.c[2] = 2 * (a.q[0] * b.q[3] + b.q[0] * a.q[3] - (a.q[1] * b.q[2] - a.q[2] * b.q[1]));
    return r;
  }
  // proj(a b^dag)
  static GL_HD Alg proj_mul_dag(const Link& a, const Link& b) { return proj_mul(a, dag(b)); }
  static GL_HD Alg proj_retr_mul_dag(const Link& a, const Link& b, T& tr) {
    tr = retr_mul_dag(a, b);
    return proj_mul_dag(a, b);
  }
  // exp(i s X), X = x.s/2: cos(|sx|/2) + i sin(|sx|/2) n.s
  static GL_HD Link expi(const Alg& x, T s) {
    T v0 = s * x.c[0], v1 = s * x.c[1], v2 = s * x.c[2];
    T th2 = v0 * v0 + v1 * v1 + v2 * v2;
    T th = sqrt(th2);
    T h = th * T(0.5);
    T sn, cs;
    sincos_r<T>(h, &sn, &cs);
    // sin(h)/th = sin(h)/(2h) with a series near 0
    T f = (h < T(1e-3)) ? T(0.5) * (T(1) - h * h / T(6) * (T(1) - h * h / T(20)))
                        : sn / th;
    Link r; r.q[0] = cs; r.q[1] = f * v0; r.q[2] = f * v1; r.q[3] = f * v2;
    return r;
  }
  template <bool TOP = false>
  static GL_HD Link expi_mul(const Alg& x, T s, const Link& u) { return mul(expi(x, s), u); }
  // pure quaternion i X = (0, x/2)
  static GL_HD Link alg_as_link(const Alg& x) { Link r; r.q[0] = 0; r.q[1] = x.c[0] / 2; r.q[2] = x.c[1] / 2; r.q[3] = x.c[2] / 2; return r; }
  static GL_HD Alg link_as_alg(const Link& m) { Alg r; r.c[0] = 2 * m.q[1]; r.c[1] = 2 * m.q[2]; r.c[2] = 2 * m.q[3]; return r; }
  // Hermitian traceless matrices M are carried as i M, which lies in the real span of
  // SU(2) (a pure quaternion), so the Link type and its products serve for them too.
  static GL_HD Link herm_from_alg(const Alg& x) { return alg_as_link(x); }
  static GL_HD Alg alg_from_herm(const Link& m) { return link_as_alg(m); }
  // U^dag X U
  static GL_HD Alg transport(const Link& u, const Alg& x) { return link_as_alg(mul(dag_mul(u, alg_as_link(x)), u)); }
  // U X U^dag
  static GL_HD Alg transport_inv(const Link& u, const Alg& x) { return link_as_alg(mul_dag(mul(u, alg_as_link(x)), u)); }
  // principal -i Log W (closed form): W = cos(th/2) + i sin(th/2) n.s -> th n
  static GL_HD Alg logi(const Link& w) {
    T s2 = w.q[1] * w.q[1] + w.q[2] * w.q[2] + w.q[3] * w.q[3];
    T s = sqrt(s2);
    T th = T(2) * atan2(s, w.q[0]);
    T f = (s < T(1e-300)) ? T(2) : th / s;
    Alg r; r.c[0] = f * w.q[1]; r.c[1] = f * w.q[2]; r.c[2] = f * w.q[3];
    return r;
  }
  static GL_HD Link reunit(const Link& m) {
    T n = sqrt(m.q[0] * m.q[0] + m.q[1] * m.q[1] + m.q[2] * m.q[2] + m.q[3] * m.q[3]);
    Link r; for (int k = 0; k < 4; ++k) r.q[k] = m.q[k] / n; return r;
  }
  // max |U^dag U - 1| and |det U - 1| for a unit quaternion: | |q|^2 - 1 |
  static GL_HD T unit_violation(const Link& m) {
    T n = m.q[0] * m.q[0] + m.q[1] * m.q[1] + m.q[2] * m.q[2] + m.q[3] * m.q[3];
    return fabs(n - T(1));
  }
};

// ----------------------------------------------------------------------------
// SU(3)
// ----------------------------------------------------------------------------

template <typename T> struct Su3 {
  static constexpr int NC = 3, NG = 8, R = 18;
  using Real = T;
  using Link = M3<T>;
  using Alg = Alg3<T>;

  static GL_HD Link zero() {
    Link r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) { r.re[i][j] = T(0); r.im[i][j] = T(0); }
    return r;
  }
  static GL_HD Link one() { Link r = zero(); r.re[0][0] = r.re[1][1] = r.re[2][2] = T(1); return r; }
  static GL_HD Alg alg_zero() { Alg r; for (int k = 0; k < 8; ++k) r.c[k] = T(0); return r; }

  // Products of 3x3 complex matrices, each entry one chain of fused multiply-adds.
  // re/im of the k-th term: (x y)  -> xr yr - xi yi, xr yi + xi yr
  //                          (x y*) -> xr yr + xi yi, xi yr - xr yi
  //                          (x* y) -> xr yr + xi yi, xr yi - xi yr
  static GL_HD Link mul(const Link& a, const Link& b) {
    Link r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        T sr = a.re[i][0] * b.re[0][j], si = a.re[i][0] * b.im[0][j];
        sr = fmx(-a.im[i][0], b.im[0][j], sr);
        si = fmx(a.im[i][0], b.re[0][j], si);
#pragma unroll
        for (int k = 1; k < 3; ++k) {
          sr = fmx(a.re[i][k], b.re[k][j], sr);
          sr = fmx(-a.im[i][k], b.im[k][j], sr);
          si = fmx(a.re[i][k], b.im[k][j], si);
          si = fmx(a.im[i][k], b.re[k][j], si);
        }
        r.re[i][j] = sr; r.im[i][j] = si;
      }
    return r;
  }
  // r (+)= a b^dag: (a b^dag)_ij = sum_k a_ik conj(b_jk)
  template <bool ACC>
  static GL_HD void mul_dag_into(Link& r, const Link& a, const Link& b) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        T sr, si;
        if (ACC) {
          sr = fmx(a.re[i][0], b.re[j][0], r.re[i][j]);
          si = fmx(a.im[i][0], b.re[j][0], r.im[i][j]);
        } else {
          sr = a.re[i][0] * b.re[j][0];
          si = a.im[i][0] * b.re[j][0];
        }
        sr = fmx(a.im[i][0], b.im[j][0], sr);
        si = fmx(-a.re[i][0], b.im[j][0], si);
#pragma unroll
        for (int k = 1; k < 3; ++k) {
          sr = fmx(a.re[i][k], b.re[j][k], sr);
          sr = fmx(a.im[i][k], b.im[j][k], sr);
          si = fmx(a.im[i][k], b.re[j][k], si);
          si = fmx(-a.re[i][k], b.im[j][k], si);
        }
        r.re[i][j] = sr; r.im[i][j] = si;
      }
  }
  // r (+)= a^dag b: (a^dag b)_ij = sum_k conj(a_ki) b_kj
  template <bool ACC>
  static GL_HD void dag_mul_into(Link& r, const Link& a, const Link& b) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        T sr, si;
        if (ACC) {
          sr = fmx(a.re[0][i], b.re[0][j], r.re[i][j]);
          si = fmx(a.re[0][i], b.im[0][j], r.im[i][j]);
        } else {
          sr = a.re[0][i] * b.re[0][j];
          si = a.re[0][i] * b.im[0][j];
        }
        sr = fmx(a.im[0][i], b.im[0][j], sr);
        si = fmx(-a.im[0][i], b.re[0][j], si);
#pragma unroll
        for (int k = 1; k < 3; ++k) {
          sr = fmx(a.re[k][i], b.re[k][j], sr);
          sr = fmx(a.im[k][i], b.im[k][j], sr);
          si = fmx(a.re[k][i], b.im[k][j], si);
          si = fmx(-a.im[k][i], b.re[k][j], si);
        }
        r.re[i][j] = sr; r.im[i][j] = si;
      }
  }
  static GL_HD Link mul_dag(const Link& a, const Link& b) { Link r; mul_dag_into<false>(r, a, b); return r; }
  static GL_HD Link dag_mul(const Link& a, const Link& b) { Link r; dag_mul_into<false>(r, a, b); return r; }
  static GL_HD void acc_mul_dag(Link& r, const Link& a, const Link& b) { mul_dag_into<true>(r, a, b); }
  static GL_HD void acc_dag_mul(Link& r, const Link& a, const Link& b) { dag_mul_into<true>(r, a, b); }
  static GL_HD void scale(Link& r, T s) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) { r.re[i][j] *= s; r.im[i][j] *= s; }
  }
  static GL_HD Link dag(const Link& a) {
    Link r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) { r.re[i][j] = a.re[j][i]; r.im[i][j] = -a.im[j][i]; }
    return r;
  }
  static GL_HD void add_to(Link& acc, const Link& a, T s) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) { acc.re[i][j] += s * a.re[i][j]; acc.im[i][j] += s * a.im[i][j]; }
  }
  // components of the hermitian traceless part of (M - M^dag)/(2i), X^a = Tr(lambda^a A)
  static GL_HD Alg proj(const Link& m) {
    const T is3 = T(0.57735026918962576451);
    Alg r;
    r.c[0] = m.im[0][1] + m.im[1][0];
    r.c[1] = m.re[0][1] - m.re[1][0];
    r.c[2] = m.im[0][0] - m.im[1][1];
    r.c[3] = m.im[0][2] + m.im[2][0];
    r.c[4] = m.re[0][2] - m.re[2][0];
    r.c[5] = m.im[1][2] + m.im[2][1];
    r.c[6] = m.re[1][2] - m.re[2][1];
    r.c[7] = (m.im[0][0] + m.im[1][1] - T(2) * m.im[2][2]) * is3;
    return r;
  }
  static GL_HD T retr(const Link& m) { return m.re[0][0] + m.re[1][1] + m.re[2][2]; }
  // proj(M) of a product M = a b or a b^dag without forming M: each off-diagonal
  // component is one fused chain over the two entries it combines, and only the
  // imaginary diagonal of M is formed (its real part drops out).
  // DAG selects b^dag: B(k, j) = b_kj, or conj(b_jk).
  template <bool DAG>
  static GL_HD void bent(const Link& b, int k, int j, T& r, T& i) {
    if (DAG) { r = b.re[j][k]; i = -b.im[j][k]; } else { r = b.re[k][j]; i = b.im[k][j]; }
  }
  // With tr given, also Re Tr M (the real diagonal, from the same products).
  template <bool DAG>
  static GL_HD Alg proj_prod(const Link& a, const Link& b, T* tr = nullptr) {
    const T is3 = T(0.57735026918962576451);
    // Im M_pq + Im M_qp and Re M_pq - Re M_qp for the pairs (0,1), (0,2), (1,2)
    T sym[3], asym[3];
    const int P[3] = {0, 0, 1}, Qd[3] = {1, 2, 2};
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      const int p = P[n], q = Qd[n];
      T y = T(0), z = T(0);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        T bkq_r, bkq_i, bkp_r, bkp_i;
        bent<DAG>(b, k, q, bkq_r, bkq_i);
        bent<DAG>(b, k, p, bkp_r, bkp_i);
        // M_pq = sum_k a_pk B_kq, M_qp = sum_k a_qk B_kp
        y = fmx(a.re[p][k], bkq_i, y);
        y = fmx(a.im[p][k], bkq_r, y);
        y = fmx(a.re[q][k], bkp_i, y);
        y = fmx(a.im[q][k], bkp_r, y);
        z = fmx(a.re[p][k], bkq_r, z);
        z = fmx(-a.im[p][k], bkq_i, z);
        z = fmx(-a.re[q][k], bkp_r, z);
        z = fmx(a.im[q][k], bkp_i, z);
      }
      sym[n] = y; asym[n] = z;
    }
    T di[3], dr[3];
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      T y = T(0), x = T(0);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        T r, i;
        bent<DAG>(b, k, p, r, i);
        y = fmx(a.re[p][k], i, y);
        y = fmx(a.im[p][k], r, y);
        if (tr) {
          x = fmx(a.re[p][k], r, x);
          x = fmx(-a.im[p][k], i, x);
        }
      }
      di[p] = y;
      dr[p] = x;
    }
    if (tr) *tr = dr[0] + dr[1] + dr[2];
    Alg r;
    r.c[0] = sym[0];
    r.c[1] = asym[0];
    r.c[2] = di[0] - di[1];
    r.c[3] = sym[1];
    r.c[4] = asym[1];
    r.c[5] = sym[2];
    r.c[6] = asym[2];
    r.c[7] = (di[0] + di[1] - T(2) * di[2]) * is3;
    return r;
  }
  static GL_HD Alg proj_mul(const Link& a, const Link& b) { return proj_prod<false>(a, b); }
  static GL_HD Alg proj_mul_dag(const Link& a, const Link& b) { return proj_prod<true>(a, b); }
  // proj(a b^dag) and Re Tr(a b^dag) together
  static GL_HD Alg proj_retr_mul_dag(const Link& a, const Link& b, T& tr) { return proj_prod<true>(a, b, &tr); }
  // hermitian matrix X = sum_a x^a lambda^a / 2, scaled by s
  static GL_HD Link herm(const Alg& x, T s) {
    const T is3 = T(0.57735026918962576451);
    T h = s * T(0.5);
    Link q;
    q.re[0][0] = h * (x.c[2] + x.c[7] * is3); q.im[0][0] = 0;
    q.re[1][1] = h * (-x.c[2] + x.c[7] * is3); q.im[1][1] = 0;
    q.re[2][2] = -h * T(2) * x.c[7] * is3; q.im[2][2] = 0;
    q.re[0][1] = h * x.c[0]; q.im[0][1] = -h * x.c[1];
    q.re[1][0] = h * x.c[0]; q.im[1][0] = h * x.c[1];
    q.re[0][2] = h * x.c[3]; q.im[0][2] = -h * x.c[4];
    q.re[2][0] = h * x.c[3]; q.im[2][0] = h * x.c[4];
    q.re[1][2] = h * x.c[5]; q.im[1][2] = -h * x.c[6];
    q.re[2][1] = h * x.c[5]; q.im[2][1] = h * x.c[6];
    return q;
  }
  // hermitian matrices are carried as themselves (3x3 complex)
  static GL_HD Link herm_from_alg(const Alg& x) { return herm(x, T(1)); }
  static GL_HD Alg alg_from_herm(const Link& m) { return alg_of_herm(m); }
  // components of a hermitian traceless matrix
  static GL_HD Alg alg_of_herm(const Link& q) {
    const T is3 = T(0.57735026918962576451);
    Alg r;
    r.c[0] = q.re[0][1] + q.re[1][0];
    r.c[1] = -q.im[0][1] + q.im[1][0];
    r.c[2] = q.re[0][0] - q.re[1][1];
    r.c[3] = q.re[0][2] + q.re[2][0];
    r.c[4] = -q.im[0][2] + q.im[2][0];
    r.c[5] = q.re[1][2] + q.re[2][1];
    r.c[6] = -q.im[1][2] + q.im[2][1];
    r.c[7] = (q.re[0][0] + q.re[1][1] - T(2) * q.re[2][2]) * is3;
    return r;
  }

  // A hermitian 3x3 matrix by its real diagonal d and the entries (0,1), (0,2), (1,2)
  // above it (real parts r, imaginary parts i); the entries below are their conjugates.
  struct Herm { T d[3], r[3], i[3]; };
  // Q = s x^a t^a
  static GL_HD Herm herm_c(const Alg& x, T s) {
    const T is3 = T(0.57735026918962576451);
    const T h = s * T(0.5);
    const T t7 = h * is3 * x.c[7], t2 = h * x.c[2];
    Herm q;
    q.d[0] = t7 + t2; q.d[1] = t7 - t2; q.d[2] = T(-2) * t7;
    q.r[0] = h * x.c[0]; q.i[0] = -h * x.c[1];
    q.r[1] = h * x.c[3]; q.i[1] = -h * x.c[4];
    q.r[2] = h * x.c[5]; q.i[2] = -h * x.c[6];
    return q;
  }

  // exp(i Q) for Q = s x^a t^a hermitian traceless.  By Cayley-Hamilton every power of
  // Q is a combination of 1, Q, Q^2 (Q^3 = c1 Q + c0 with c0 = det Q, c1 = Tr Q^2 / 2),
  // so exp(iQ) = h0 + h1 Q + h2 Q^2 with complex scalars h.  They are obtained by
  // scaling and squaring in that coefficient space: the exponential series of Q / 2^k
  // (spectral radius <= 1/2, sqrt(4 c1 / 3) bounds it) is summed to a remainder below
  // the unit roundoff (14 terms in double, 8 in float), and each of the k squarings
  // (h0 + h1 Q + h2 Q^2)^2 is reduced with the same identity.  Exact to rounding; no
  // transcendental functions and no branches on the data apart from k.  Returns
  // exp(iQ) as a matrix (hermitian structure of Q and Q^2 used throughout).
  static GL_HD Link expi(const Alg& x, T s) {
    const Herm q = herm_c(x, s);
    // P = Q^2
    const T n0 = fmx(q.r[0], q.r[0], q.i[0] * q.i[0]);
    const T n1 = fmx(q.r[1], q.r[1], q.i[1] * q.i[1]);
    const T n2 = fmx(q.r[2], q.r[2], q.i[2] * q.i[2]);
    Herm p;
    p.d[0] = fmx(q.d[0], q.d[0], n0 + n1);
    p.d[1] = fmx(q.d[1], q.d[1], n0 + n2);
    p.d[2] = fmx(q.d[2], q.d[2], n1 + n2);
    const T s01 = q.d[0] + q.d[1], s02 = q.d[0] + q.d[2], s12 = q.d[1] + q.d[2];
    p.r[0] = fmx(q.r[0], s01, fmx(q.r[1], q.r[2], q.i[1] * q.i[2]));
    p.i[0] = fmx(q.i[0], s01, fmx(q.i[1], q.r[2], -q.r[1] * q.i[2]));
    p.r[1] = fmx(q.r[1], s02, fmx(q.r[0], q.r[2], -q.i[0] * q.i[2]));
    p.i[1] = fmx(q.i[1], s02, fmx(q.r[0], q.i[2], q.i[0] * q.r[2]));
    p.r[2] = fmx(q.r[2], s12, fmx(q.r[0], q.r[1], q.i[0] * q.i[1]));
    p.i[2] = fmx(q.i[2], s12, fmx(q.r[0], q.i[1], -q.i[0] * q.r[1]));
    const T c1 = T(0.5) * (p.d[0] + p.d[1] + p.d[2]);
    // c0 = det Q = d0 d1 d2 - d0 |q12|^2 - d1 |q02|^2 - d2 |q01|^2 + 2 Re(q01 q12 conj(q02))
    const T acr = fmx(q.r[0], q.r[2], -q.i[0] * q.i[2]), aci = fmx(q.r[0], q.i[2], q.i[0] * q.r[2]);
    T c0 = q.d[0] * q.d[1] * q.d[2];
    c0 = fmx(-q.d[0], n2, c0);
    c0 = fmx(-q.d[1], n1, c0);
    c0 = fmx(-q.d[2], n0, c0);
    c0 = fmx(T(2), fmx(acr, q.r[1], aci * q.i[1]), c0);
    // scaling: k halvings bring the spectral radius bound below 1/2.  The count is capped
    // at what the largest finite value needs (r2 < 2^1024 in double, 2^128 in float), so an
    // infinite input ends the loop too (its result is non-finite, and reported as such).
    T r2 = T(4) / T(3) * c1;       // bound on the squared spectral radius
    int k = 0;
    T sc = T(1);
    constexpr int KMAX = sizeof(T) == 8 ? 600 : 80;
    while (r2 > T(0.25) && k < KMAX) { r2 *= T(0.25); sc *= T(0.5); ++k; }
    const T c0k = c0 * sc * sc * sc, c1k = c1 * sc * sc;
    // series of exp(i Q_k), Q_k^n = a + b Q_k + c Q_k^2
    constexpr int NT = sizeof(T) == 8 ? 14 : 8;
    T a = T(1), b = T(0), c = T(0);
    T g0r = T(1), g0i = T(0), g1r = T(0), g1i = T(0), g2r = T(0), g2i = T(0);
    T w = T(1);
#pragma unroll
    for (int n = 1; n <= NT; ++n) {
      const T an = c0k * c, bn = fmx(c1k, c, a), cn = b;
      a = an; b = bn; c = cn;
      w /= T(n);
      // i^n: 1, i, -1, -i
      const T ws = ((n & 3) < 2) ? w : -w;
      if (n & 1) { g0i = fmx(ws, a, g0i); g1i = fmx(ws, b, g1i); g2i = fmx(ws, c, g2i); }
      else { g0r = fmx(ws, a, g0r); g1r = fmx(ws, b, g1r); g2r = fmx(ws, c, g2r); }
    }
    // coefficients with respect to Q
    T h0r = g0r, h0i = g0i, h1r = g1r * sc, h1i = g1i * sc, h2r = g2r * sc * sc, h2i = g2i * sc * sc;
    for (int m = 0; m < k; ++m) {
      // n0 = h0^2 + 2 h1 h2 c0, n1 = 2 h0 h1 + 2 h1 h2 c1 + h2^2 c0, n2 = h1^2 + 2 h0 h2 + h2^2 c1
      const T h00r = h0r * h0r - h0i * h0i, h00i = T(2) * h0r * h0i;
      const T h12r = h1r * h2r - h1i * h2i, h12i = h1r * h2i + h1i * h2r;
      const T h01r = h0r * h1r - h0i * h1i, h01i = h0r * h1i + h0i * h1r;
      const T h22r = h2r * h2r - h2i * h2i, h22i = T(2) * h2r * h2i;
      const T h11r = h1r * h1r - h1i * h1i, h11i = T(2) * h1r * h1i;
      const T h02r = h0r * h2r - h0i * h2i, h02i = h0r * h2i + h0i * h2r;
      h0r = h00r + T(2) * c0 * h12r; h0i = h00i + T(2) * c0 * h12i;
      h1r = T(2) * h01r + T(2) * c1 * h12r + c0 * h22r; h1i = T(2) * h01i + T(2) * c1 * h12i + c0 * h22i;
      h2r = h11r + T(2) * h02r + c1 * h22r; h2i = h11i + T(2) * h02i + c1 * h22i;
    }
    // R = h0 + h1 Q + h2 Q^2
    Link R;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      R.re[d][d] = fmx(h1r, q.d[d], fmx(h2r, p.d[d], h0r));
      R.im[d][d] = fmx(h1i, q.d[d], fmx(h2i, p.d[d], h0i));
    }
    const int UP[3] = {0, 0, 1}, LO[3] = {1, 2, 2};
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      const T A = fmx(h1r, q.r[n], h2r * p.r[n]);
      const T B = fmx(h1i, q.i[n], h2i * p.i[n]);
      const T C = fmx(h1r, q.i[n], h2r * p.i[n]);
      const T D = fmx(h1i, q.r[n], h2i * p.r[n]);
      R.re[UP[n]][LO[n]] = A - B; R.im[UP[n]][LO[n]] = C + D;
      R.re[LO[n]][UP[n]] = A + B; R.im[LO[n]][UP[n]] = D - C;
    }
    return R;
  }
  // exp(i s X) u; with TOP only rows 0 and 1 are formed (row 2 is set to zero), which
  // is all that the two-row link storage keeps.
  template <bool TOP = false>
  static GL_HD Link expi_mul(const Alg& x, T s, const Link& u) {
    const Link R = expi(x, s);
    Link r;
    constexpr int NR = TOP ? 2 : 3;
#pragma unroll
    for (int i = 0; i < NR; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        T sr = R.re[i][0] * u.re[0][j], si = R.re[i][0] * u.im[0][j];
        sr = fmx(-R.im[i][0], u.im[0][j], sr);
        si = fmx(R.im[i][0], u.re[0][j], si);
#pragma unroll
        for (int k = 1; k < 3; ++k) {
          sr = fmx(R.re[i][k], u.re[k][j], sr);
          sr = fmx(-R.im[i][k], u.im[k][j], sr);
          si = fmx(R.re[i][k], u.im[k][j], si);
          si = fmx(R.im[i][k], u.re[k][j], si);
        }
        r.re[i][j] = sr; r.im[i][j] = si;
      }
    if (TOP)
#pragma unroll
      for (int j = 0; j < 3; ++j) { r.re[2][j] = T(0); r.im[2][j] = T(0); }
    return r;
  }
  // U^dag X U
  // Components of M = W X V for hermitian X = x^a t^a, with (W, V) = (u^dag, u) (INV
  // false) or (u, u^dag) (INV true).  M is hermitian, so only its upper triangle and the
  // real part of its diagonal are formed: Y = X V uses the real diagonal of X, then
  // M_pq = sum_k W_pk Y_kq for p <= q.
  template <bool INV>
  static GL_HD Alg sandwich(const Link& u, const Alg& x) {
    const Herm q = herm_c(x, T(1));
    // X entries: X_pp = d_p, X_pq = r + i im above the diagonal, conjugate below
    const int UP[3][3] = {{-1, 0, 1}, {0, -1, 2}, {1, 2, -1}};
    auto vr = [&](int k, int j) { return INV ? u.re[j][k] : u.re[k][j]; };
    auto vi = [&](int k, int j) { return INV ? -u.im[j][k] : u.im[k][j]; };
    auto wr = [&](int p, int k) { return INV ? u.re[p][k] : u.re[k][p]; };
    auto wi = [&](int p, int k) { return INV ? u.im[p][k] : -u.im[k][p]; };
    T yr[3][3], yi[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        T sr = q.d[i] * vr(i, j), si = q.d[i] * vi(i, j);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          if (k == i) continue;
          const int n = UP[i][k];
          const T xr = q.r[n], xi = i < k ? q.i[n] : -q.i[n];
          sr = fmx(xr, vr(k, j), sr);
          sr = fmx(-xi, vi(k, j), sr);
          si = fmx(xr, vi(k, j), si);
          si = fmx(xi, vr(k, j), si);
        }
        yr[i][j] = sr; yi[i][j] = si;
      }
    T mr[3][3], mi[3][3];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int j = p; j < 3; ++j) {
        T sr = T(0), si = T(0);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          sr = fmx(wr(p, k), yr[k][j], sr);
          sr = fmx(-wi(p, k), yi[k][j], sr);
          if (j != p) {
            si = fmx(wr(p, k), yi[k][j], si);
            si = fmx(wi(p, k), yr[k][j], si);
          }
        }
        mr[p][j] = sr; mi[p][j] = si;
      }
    const T is3 = T(0.57735026918962576451);
    Alg r;
    r.c[0] = T(2) * mr[0][1];
    r.c[1] = T(-2) * mi[0][1];
    r.c[2] = mr[0][0] - mr[1][1];
    r.c[3] = T(2) * mr[0][2];
    r.c[4] = T(-2) * mi[0][2];
    r.c[5] = T(2) * mr[1][2];
    r.c[6] = T(-2) * mi[1][2];
    r.c[7] = (mr[0][0] + mr[1][1] - T(2) * mr[2][2]) * is3;
    return r;
  }
  // U^dag X U
  static GL_HD Alg transport(const Link& u, const Alg& x) { return sandwich<false>(u, x); }
  // U X U^dag
  static GL_HD Alg transport_inv(const Link& u, const Alg& x) { return sandwich<true>(u, x); }
  // principal -i Log W for W close to 1 (all eigen-angles well inside (-pi/2, pi/2)):
  // fixed point of H <- H + proj(exp(-iH/2) W exp(-iH/2)), which converges with the
  // cube of the symmetric-splitting error; at the fixed point W = exp(iH).
  static GL_HD Alg logi(const Link& w) {
    Alg h = proj(w);
    for (int it = 0; it < 40; ++it) {
      Link hm = expi(h, T(-0.5));
      Link R = mul(mul(hm, w), hm);
      Alg d = proj(R);
      T n = T(0);
      for (int k = 0; k < 8; ++k) { h.c[k] += d.c[k]; n += d.c[k] * d.c[k]; }
      if (n < (sizeof(T) == 8 ? T(1e-30) : T(1e-14))) break;
    }
    return h;
  }
  // rows 1, 2 Gram-Schmidt, row 3 = conj(r1 x r2)
  static GL_HD Link reunit(const Link& m) {
    Link r = m;
    T n0 = T(0);
    for (int k = 0; k < 3; ++k) n0 += r.re[0][k] * r.re[0][k] + r.im[0][k] * r.im[0][k];
    n0 = T(1) / sqrt(n0);
    for (int k = 0; k < 3; ++k) { r.re[0][k] *= n0; r.im[0][k] *= n0; }
    // r1 -= (r0^* . r1) r0
    T pr = 0, pi = 0;
    for (int k = 0; k < 3; ++k) {
      pr += r.re[0][k] * r.re[1][k] + r.im[0][k] * r.im[1][k];
      pi += r.re[0][k] * r.im[1][k] - r.im[0][k] * r.re[1][k];
    }
    for (int k = 0; k < 3; ++k) {
      r.re[1][k] -= pr * r.re[0][k] - pi * r.im[0][k];
      r.im[1][k] -= pr * r.im[0][k] + pi * r.re[0][k];
    }
    T n1 = T(0);
    for (int k = 0; k < 3; ++k) n1 += r.re[1][k] * r.re[1][k] + r.im[1][k] * r.im[1][k];
    n1 = T(1) / sqrt(n1);
    for (int k = 0; k < 3; ++k) { r.re[1][k] *= n1; r.im[1][k] *= n1; }
    // r2 = conj(r0 x r1)
    for (int k = 0; k < 3; ++k) {
      int a = (k + 1) % 3, b = (k + 2) % 3;
      T cr = r.re[0][a] * r.re[1][b] - r.im[0][a] * r.im[1][b] - (r.re[0][b] * r.re[1][a] - r.im[0][b] * r.im[1][a]);
      T ci = r.re[0][a] * r.im[1][b] + r.im[0][a] * r.re[1][b] - (r.re[0][b] * r.im[1][a] + r.im[0][b] * r.re[1][a]);
      r.re[2][k] = cr; r.im[2][k] = -ci;
    }
    return r;
  }
  // max |U^dag U - 1|_entry and |det U - 1|
  static GL_HD T unit_violation(const Link& m) {
    Link p = dag_mul(m, m);
    T v = T(0);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        T d = fabs(p.re[i][j] - (i == j ? T(1) : T(0)));
        T e = fabs(p.im[i][j]);
        v = d > v ? d : v; v = e > v ? e : v;
      }
    // det
    T dr = 0, di = 0;
    for (int k = 0; k < 3; ++k) {
      int a = (k + 1) % 3, b = (k + 2) % 3;
      // cofactor of (0,k): m1a m2b - m1b m2a
      T cr = m.re[1][a] * m.re[2][b] - m.im[1][a] * m.im[2][b] - (m.re[1][b] * m.re[2][a] - m.im[1][b] * m.im[2][a]);
      T ci = m.re[1][a] * m.im[2][b] + m.im[1][a] * m.re[2][b] - (m.re[1][b] * m.im[2][a] + m.im[1][b] * m.re[2][a]);
      dr += m.re[0][k] * cr - m.im[0][k] * ci;
      di += m.re[0][k] * ci + m.im[0][k] * cr;
    }
    T dd = sqrt((dr - 1) * (dr - 1) + di * di);
    return dd > v ? dd : v;
  }
};

template <int NC, typename T> struct GroupOf;
template <typename T> struct GroupOf<2, T> { using type = Su2<T>; };
template <typename T> struct GroupOf<3, T> { using type = Su3<T>; };

}  // namespace gl
