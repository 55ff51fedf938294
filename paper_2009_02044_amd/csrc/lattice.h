// Lattice geometry and structure-of-arrays field access.
//
// Site index s = (z * nt + y) * nt + x, x fastest, so a wavefront of 64 lanes reads
// 64 consecutive x.  Every real component of every field is its own contiguous
// array of V values:
//   links  U[(i * R + c) * V + s]     i = direction (0:x 1:y 2:z), c = 0..R-1
//          SU(2): c = quaternion component; SU(3): c = 2 (3 r + k) + {0 re, 1 im}
//   E      E[(i * NG + a) * V + s]    algebra components E^a = 2 Tr(t^a E)
//   rho    rho[a * V + s]
// All three directions are periodic.
#pragma once
#include <stdint.h>
#include "group.h"

namespace gl {

struct Geom {
  int nt, nz;
  int64_t V;     // nt * nt * nz
  int64_t layer; // nt * nt
};

GL_HD int wrap_add(int v, int d, int n) {
  int r = v + d;
  r = r >= n ? r - n : r;
  r = r < 0 ? r + n : r;
  return r;
}

struct Site {
  int x, y, z;
};

GL_HD int64_t site_index(const Geom& g, int x, int y, int z) {
  return ((int64_t)z * g.nt + y) * g.nt + x;
}

// coordinates of x + d e_i
GL_HD Site shifted(const Geom& g, Site s, int i, int d) {
  if (i == 0) s.x = wrap_add(s.x, d, g.nt);
  else if (i == 1) s.y = wrap_add(s.y, d, g.nt);
  else s.z = wrap_add(s.z, d, g.nz);
  return s;
}

GL_HD int64_t idx(const Geom& g, Site s) { return site_index(g, s.x, s.y, s.z); }

// ---- link load / store (storage type S, compute type T) --------------------
template <typename T, typename S>
GL_HD void load_link(Q2<T>& l, const S* __restrict__ U, int i, int64_t s, int64_t V) {
  const S* p = U + (int64_t)(i * 4) * V + s;
#pragma unroll
  for (int c = 0; c < 4; ++c) l.q[c] = (T)p[c * V];
}
template <typename T, typename S>
GL_HD void store_link(const Q2<T>& l, S* __restrict__ U, int i, int64_t s, int64_t V) {
  S* p = U + (int64_t)(i * 4) * V + s;
#pragma unroll
  for (int c = 0; c < 4; ++c) p[c * V] = (S)l.q[c];
}
template <typename T, typename S>
GL_HD void load_link(M3<T>& l, const S* __restrict__ U, int i, int64_t s, int64_t V) {
  const S* p = U + (int64_t)(i * 18) * V + s;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      l.re[r][k] = (T)p[(2 * (3 * r + k)) * V];
      l.im[r][k] = (T)p[(2 * (3 * r + k) + 1) * V];
    }
}
template <typename T, typename S>
GL_HD void store_link(const M3<T>& l, S* __restrict__ U, int i, int64_t s, int64_t V) {
  S* p = U + (int64_t)(i * 18) * V + s;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      p[(2 * (3 * r + k)) * V] = (S)l.re[r][k];
      p[(2 * (3 * r + k) + 1) * V] = (S)l.im[r][k];
    }
}

// ---- algebra load / store: base points at component 0 of the wanted direction --
template <typename A, typename S>
GL_HD void load_alg(A& a, const S* __restrict__ base, int64_t s, int64_t V) {
  constexpr int NG = sizeof(a.c) / sizeof(a.c[0]);
#pragma unroll
  for (int k = 0; k < NG; ++k) a.c[k] = (decltype(a.c[0] + 0))base[k * V + s];
}
template <typename A, typename S>
GL_HD void store_alg(const A& a, S* __restrict__ base, int64_t s, int64_t V) {
  constexpr int NG = sizeof(a.c) / sizeof(a.c[0]);
#pragma unroll
  for (int k = 0; k < NG; ++k) base[k * V + s] = (S)a.c[k];
}

// Per-step constants shared by the kernels.
struct StepConst {
  double a[3];       // lattice spacings a_x = a_y = a_T, a_z = a_L
  double dt;
  int hop;           // 1 on a step where every charge advances one cell
  int offA, offB;    // co-moving storage offsets of the two charge populations
};

// Co-moving charge storage: nucleus B (moving +z) keeps the charge that sits at
// physical layer z in slot (z - offB) mod nz; nucleus A (moving -z) in slot
// (z + offA) mod nz.  A hop then only increments the offsets: the parallel
// transport that goes with it rewrites each slot in place.
GL_HD int slotB(int z, int off, int nz) { int r = (z - off) % nz; return r < 0 ? r + nz : r; }
GL_HD int slotA(int z, int off, int nz) { return (z + off) % nz; }

}  // namespace gl
