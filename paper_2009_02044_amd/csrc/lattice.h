// Lattice geometry and tiled structure-of-arrays field access.
//
// Site index s = (z * nt + y) * nt + x, x fastest, so a wavefront of 64 lanes reads
// 64 consecutive x.  Fields are stored per direction as arrays of records: the sites
// are grouped in blocks of B = 128 / sizeof(real) consecutive sites (16 in double,
// 32 in float) and a record holds, for one block, each real component as a row of
// B values (one 128-byte line).  A wavefront reading component c of 64 consecutive
// sites touches whole 128-byte lines, and all components of one site are at fixed
// offsets c * 128 bytes from the site's address, so one 64-bit address per
// (site, direction) serves every component through immediate offsets.
//   links  direction i: record width R (SU(2): 4 quaternion reals; SU(3): 18 reals,
//          c = 2 (3 r + k) + {0 re, 1 im})
//   E      direction i: record width NG (algebra components E^a = 2 Tr(t^a E))
//   rho    record width NG
// The site count is padded to Vp (a multiple of 32) and direction i of a field
// starts at element i * Vp * width.  All three lattice directions are periodic.
#pragma once
#include <stdint.h>
#include "group.h"

namespace gl {

struct Geom {
  int nt, nz;
  int64_t V;     // nt * nt * nz
  int64_t Vp;    // V rounded up to a multiple of 32 (record padding)
  int64_t layer; // nt * nt
};

constexpr int VPAD = 32;
GL_HD int64_t padded_sites(int64_t V) { return (V + VPAD - 1) / VPAD * VPAD; }

GL_HD int wrap_add(int v, int d, int n) {
  int r = v + d;
  r = r >= n ? r - n : r;
  r = r < 0 ? r + n : r;
  return r;
}

struct Site {
  int x, y, z;
};

// Lattices hold fewer than 2^31 sites, so site indices are 32-bit.
GL_HD uint32_t site_index(const Geom& g, int x, int y, int z) {
  return ((uint32_t)z * (uint32_t)g.nt + (uint32_t)y) * (uint32_t)g.nt + (uint32_t)x;
}

// coordinates of x + d e_i
GL_HD Site shifted(const Geom& g, Site s, int i, int d) {
  if (i == 0) s.x = wrap_add(s.x, d, g.nt);
  else if (i == 1) s.y = wrap_add(s.y, d, g.nt);
  else s.z = wrap_add(s.z, d, g.nz);
  return s;
}

GL_HD uint32_t idx(const Geom& g, Site s) { return site_index(g, s.x, s.y, s.z); }

// ---- tiled record access ----------------------------------------------------
template <typename S> struct Rec {
  static constexpr int B = 128 / (int)sizeof(S);          // sites per block
  static constexpr int LOGB = sizeof(S) == 8 ? 4 : 5;
};
// byte offset of site s inside one direction's array of records of width W
template <typename S, int W> GL_HD uint64_t rec_off(uint32_t s) {
  return (uint64_t)(s >> Rec<S>::LOGB) * (uint64_t)(W * 128) + (uint64_t)((s & (Rec<S>::B - 1)) * sizeof(S));
}
// element index of (direction-local component c, site s) for width W (host transfers)
template <typename S> GL_HD int64_t rec_elem(int64_t s, int c, int W) {
  return (s >> Rec<S>::LOGB) * (int64_t)(W * Rec<S>::B) + (int64_t)c * Rec<S>::B + (s & (Rec<S>::B - 1));
}

template <typename S> GL_HD const S* field_dir(const S* f, int i, int W, int64_t Vp) { return f + (int64_t)i * Vp * W; }
template <typename S> GL_HD S* field_dir(S* f, int i, int W, int64_t Vp) { return f + (int64_t)i * Vp * W; }

template <typename S> GL_HD const S& at(const char* p, int c) { return *(const S*)(p + c * 128); }
template <typename S> GL_HD S& at(char* p, int c) { return *(S*)(p + c * 128); }

// ---- link load / store (storage type S, compute type T); Vp = padded site count --
template <typename T, typename S>
GL_HD void load_link(Q2<T>& l, const S* __restrict__ U, int i, uint32_t s, int64_t Vp) {
  const char* p = (const char*)field_dir(U, i, 4, Vp) + rec_off<S, 4>(s);
#pragma unroll
  for (int c = 0; c < 4; ++c) l.q[c] = (T)at<S>(p, c);
}
template <typename T, typename S>
GL_HD void store_link(const Q2<T>& l, S* __restrict__ U, int i, uint32_t s, int64_t Vp) {
  char* p = (char*)field_dir(U, i, 4, Vp) + rec_off<S, 4>(s);
#pragma unroll
  for (int c = 0; c < 4; ++c) at<S>(p, c) = (S)l.q[c];
}
template <typename T, typename S>
GL_HD void load_link(M3<T>& l, const S* __restrict__ U, int i, uint32_t s, int64_t Vp) {
  const char* p = (const char*)field_dir(U, i, 18, Vp) + rec_off<S, 18>(s);
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      l.re[r][k] = (T)at<S>(p, 2 * (3 * r + k));
      l.im[r][k] = (T)at<S>(p, 2 * (3 * r + k) + 1);
    }
}
template <typename T, typename S>
GL_HD void store_link(const M3<T>& l, S* __restrict__ U, int i, uint32_t s, int64_t Vp) {
  char* p = (char*)field_dir(U, i, 18, Vp) + rec_off<S, 18>(s);
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      at<S>(p, 2 * (3 * r + k)) = (S)l.re[r][k];
      at<S>(p, 2 * (3 * r + k) + 1) = (S)l.im[r][k];
    }
}

// ---- algebra load / store: f = field base, i = direction (0 for rho) ----------
template <typename A, typename S>
GL_HD void load_alg(A& a, const S* __restrict__ f, int i, uint32_t s, int64_t Vp) {
  constexpr int NG = sizeof(a.c) / sizeof(a.c[0]);
  const char* p = (const char*)field_dir(f, i, NG, Vp) + rec_off<S, NG>(s);
#pragma unroll
  for (int k = 0; k < NG; ++k) a.c[k] = (decltype(a.c[0] + 0))at<S>(p, k);
}
template <typename A, typename S>
GL_HD void store_alg(const A& a, S* __restrict__ f, int i, uint32_t s, int64_t Vp) {
  constexpr int NG = sizeof(a.c) / sizeof(a.c[0]);
  char* p = (char*)field_dir(f, i, NG, Vp) + rec_off<S, NG>(s);
#pragma unroll
  for (int k = 0; k < NG; ++k) at<S>(p, k) = (S)a.c[k];
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
