// Lattice geometry and tiled structure-of-arrays field access.
//
// Site index s = (z * nt + y) * nt + x, x fastest, so a wavefront of 64 lanes reads
// 64 consecutive x.  Each field direction is an array of records of 64 consecutive
// sites; inside a record the real components are grouped in 16-byte chunks, one row
// of 64 chunks per group (see the record access below), so every lane fetches a
// link or an algebra element with few 16-byte loads and a wavefront's load covers a
// contiguous 1 KiB.
//   links  direction i: SU(2): 4 quaternion reals; SU(3): rows 0 and 1, 12 reals,
//          c = 2 (3 r + k) + {0 re, 1 im} (row 2 is rebuilt on load, see load_link)
//   E      direction i: width NG (algebra components E^a = 2 Tr(t^a E))
//   rho    width NG
// The site count is padded to Vp (a multiple of 64) and direction i of a field
// starts at element i * Vp * width.  All three lattice directions are periodic.
#pragma once
#include <stdint.h>
#include "group.h"

namespace gl {

struct Geom {
  int nt, nz;
  int64_t V;     // nt * nt * nz
  int64_t Vp;    // V rounded up to a multiple of 64 (record padding)
  int64_t layer; // nt * nt
};

constexpr int VPAD = 64;
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
// A record holds RB = 64 consecutive sites of one direction.  Inside a record the
// components are grouped in 16-byte chunks (4 floats or 2 doubles): chunk row q
// stores components [q VW, q VW + VW) of all 64 sites, 16 bytes per site, so one
// 16-byte load per lane fetches VW components and a wavefront reads a contiguous
// 1 KiB row.  Components left over (W mod VW) form a last, narrower row.
constexpr int RB = 64;
template <typename S> struct Rec {
  static constexpr int VW = 16 / (int)sizeof(S);          // components per 16-byte chunk
};
template <typename S, int W> struct RecShape {
  static constexpr int VW = Rec<S>::VW;
  static constexpr int NF = W / VW;                        // full 16-byte rows
  static constexpr int TL = W % VW;                        // components in the last row
  static constexpr uint32_t BYTES = RB * W * sizeof(S);   // record size
};
// element index of (component c, site s) in one direction's array of width W (host transfers)
template <typename S> GL_HD int64_t rec_elem(int64_t s, int c, int W) {
  const int VW = Rec<S>::VW, nf = W / VW, tl = W % VW;
  const int64_t rec = (s / RB) * (int64_t)RB * W;
  const int l = (int)(s % RB);
  if (c < nf * VW) return rec + (int64_t)(c / VW) * RB * VW + (int64_t)l * VW + c % VW;
  return rec + (int64_t)nf * RB * VW + (int64_t)l * tl + (c - nf * VW);
}

template <typename S> GL_HD const S* field_dir(const S* f, int i, int W, int64_t Vp) { return f + (int64_t)i * Vp * W; }
template <typename S> GL_HD S* field_dir(S* f, int i, int W, int64_t Vp) { return f + (int64_t)i * Vp * W; }

template <typename S> struct Vec16;
template <> struct Vec16<float> { using type = float4; };
template <> struct Vec16<double> { using type = double2; };

template <typename S> struct NVec16;
template <> struct NVec16<float> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct NVec16<double> { typedef double type __attribute__((ext_vector_type(2))); };

// load / store the W components of site s from one direction's record array.  NT marks
// the loads non-temporal: for fields that only the site's own thread reads (E, the
// charges), so that they leave the L2 to the links the neighbours still read.
#ifndef GL_NT_LOAD
#define GL_NT_LOAD 1
#endif
template <typename T, typename S, int W, bool NT = false>
GL_HD void load_comps(T (&v)[W], const S* __restrict__ dir, uint32_t s) {
  using Sh = RecShape<S, W>;
  using NV = typename NVec16<S>::type;
  const char* rec = (const char*)dir + (uint64_t)(s / RB) * Sh::BYTES;
  const uint32_t l = s % RB;
#pragma unroll
  for (int q = 0; q < Sh::NF; ++q) {
    const NV* src = (const NV*)(rec + q * (RB * 16) + l * 16);
    NV x;
#if GL_NT_LOAD && defined(__HIP_DEVICE_COMPILE__)
    if constexpr (NT) x = __builtin_nontemporal_load(src);
    else x = *src;
#else
    x = *src;
#endif
#pragma unroll
    for (int k = 0; k < Sh::VW; ++k) v[q * Sh::VW + k] = (T)x[k];
  }
  if constexpr (Sh::TL > 0) {
    const S* t = (const S*)(rec + Sh::NF * (RB * 16) + l * (Sh::TL * sizeof(S)));
#pragma unroll
    for (int k = 0; k < Sh::TL; ++k) v[Sh::NF * Sh::VW + k] = (T)t[k];
  }
}
// Stores of kernel outputs are marked non-temporal (streamed past the caches) unless
// GL_NT_STORE is 0: no kernel reads back what it writes, and the stream would
// otherwise displace the neighbour links that other work-groups still read.
#ifndef GL_NT_STORE
#define GL_NT_STORE 1
#endif
template <typename T, typename S, int W>
GL_HD void store_comps(const T (&v)[W], S* __restrict__ dir, uint32_t s) {
  using Sh = RecShape<S, W>;
  using NV = typename NVec16<S>::type;
  char* rec = (char*)dir + (uint64_t)(s / RB) * Sh::BYTES;
  const uint32_t l = s % RB;
#pragma unroll
  for (int q = 0; q < Sh::NF; ++q) {
    NV x;
#pragma unroll
    for (int k = 0; k < Sh::VW; ++k) x[k] = (S)v[q * Sh::VW + k];
    NV* dst = (NV*)(rec + q * (RB * 16) + l * 16);
#if GL_NT_STORE && defined(__HIP_DEVICE_COMPILE__)
    __builtin_nontemporal_store(x, dst);
#else
    *dst = x;
#endif
  }
  if constexpr (Sh::TL > 0) {
    S* t = (S*)(rec + Sh::NF * (RB * 16) + l * (Sh::TL * sizeof(S)));
#pragma unroll
    for (int k = 0; k < Sh::TL; ++k) t[k] = (S)v[Sh::NF * Sh::VW + k];
  }
}

// ---- link load / store (storage type S, compute type T); Vp = padded site count --
template <typename T, typename S>
GL_HD void load_link(Q2<T>& l, const S* __restrict__ U, int i, uint32_t s, int64_t Vp) {
  load_comps<T, S, 4>(l.q, field_dir(U, i, 4, Vp), s);
}
template <typename T, typename S>
GL_HD void store_link(const Q2<T>& l, S* __restrict__ U, int i, uint32_t s, int64_t Vp) {
  store_comps<T, S, 4>(l.q, field_dir(U, i, 4, Vp), s);
}
// Row 2 of a special unitary matrix from rows 0 and 1: u_2k = conj(u_0a u_1b - u_0b u_1a),
// (a, b) = (k+1, k+2) mod 3; each real part one fused chain.
template <typename T>
GL_HD void complete_row2(M3<T>& l) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int a = (k + 1) % 3, b = (k + 2) % 3;
    T cr = l.re[0][a] * l.re[1][b];
    cr = fmx(-l.im[0][a], l.im[1][b], cr);
    cr = fmx(-l.re[0][b], l.re[1][a], cr);
    cr = fmx(l.im[0][b], l.im[1][a], cr);
    T ci = l.re[0][a] * l.im[1][b];
    ci = fmx(l.im[0][a], l.re[1][b], ci);
    ci = fmx(-l.re[0][b], l.im[1][a], ci);
    ci = fmx(-l.im[0][b], l.re[1][a], ci);
    l.re[2][k] = cr;
    l.im[2][k] = -ci;
  }
}
// SU(3) links are stored by their first two rows (12 reals, c = 2 (3 r + k) + {re, im},
// r = 0, 1); for a special unitary matrix the third row is conj(row 0 x row 1), rebuilt on
// every load.  A third fewer bytes and load instructions than the full matrix.
constexpr int SU3_STORED = 12;
template <typename T, typename S>
GL_HD void load_link(M3<T>& l, const S* __restrict__ U, int i, uint32_t s, int64_t Vp) {
  T v[SU3_STORED];
  load_comps<T, S, SU3_STORED>(v, field_dir(U, i, SU3_STORED, Vp), s);
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      l.re[r][k] = v[2 * (3 * r + k)];
      l.im[r][k] = v[2 * (3 * r + k) + 1];
    }
  complete_row2(l);
}
// link from its stored reals (SU(3): rows 0 and 1, row 2 rebuilt)
template <typename T> GL_HD void link_from_stored(Q2<T>& l, const T (&v)[4]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) l.q[k] = v[k];
}
template <typename T> GL_HD void link_from_stored(M3<T>& l, const T (&v)[SU3_STORED]) {
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      l.re[r][k] = v[2 * (3 * r + k)];
      l.im[r][k] = v[2 * (3 * r + k) + 1];
    }
  complete_row2(l);
}
template <typename T, typename S>
GL_HD void store_link(const M3<T>& l, S* __restrict__ U, int i, uint32_t s, int64_t Vp) {
  T v[SU3_STORED];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      v[2 * (3 * r + k)] = l.re[r][k];
      v[2 * (3 * r + k) + 1] = l.im[r][k];
    }
  store_comps<T, S, SU3_STORED>(v, field_dir(U, i, SU3_STORED, Vp), s);
}
// stored reals per link
template <typename L> struct StoredWidth;
template <typename T> struct StoredWidth<Q2<T>> { static constexpr int value = 4; };
template <typename T> struct StoredWidth<M3<T>> { static constexpr int value = SU3_STORED; };

// ---- algebra load / store: f = field base, i = direction (0 for rho) ----------
template <typename A, typename S>
GL_HD void load_alg(A& a, const S* __restrict__ f, int i, uint32_t s, int64_t Vp) {
  constexpr int NG = sizeof(a.c) / sizeof(a.c[0]);
  load_comps<decltype(a.c[0] + 0), S, NG>(a.c, field_dir(f, i, NG, Vp), s);
}
// the same for a field only the site's own thread reads (non-temporal loads)
template <typename A, typename S>
GL_HD void load_alg_own(A& a, const S* __restrict__ f, int i, uint32_t s, int64_t Vp) {
  constexpr int NG = sizeof(a.c) / sizeof(a.c[0]);
  load_comps<decltype(a.c[0] + 0), S, NG, true>(a.c, field_dir(f, i, NG, Vp), s);
}
template <typename A, typename S>
GL_HD void store_alg(const A& a, S* __restrict__ f, int i, uint32_t s, int64_t Vp) {
  constexpr int NG = sizeof(a.c) / sizeof(a.c[0]);
  store_comps<decltype(a.c[0] + 0), S, NG>(a.c, field_dir(f, i, NG, Vp), s);
}

// Work-group placement: the hardware hands work-groups to the 8 XCDs round-robin
// (b mod 8), and each XCD has its own L2.  Renumbering so that XCD k receives one
// contiguous range of blocks keeps the y and z neighbours of a block in the same L2.
// The map is a bijection of [0, nb) for any nb.
constexpr int NXCD = 8;
GL_HD uint32_t xcd_remap(uint32_t b, uint32_t nb) {
  const uint32_t q = nb / NXCD, r = nb % NXCD, x = b % NXCD;
  return x * q + (x < r ? x : r) + b / NXCD;
}
// The same in chunks of C consecutive indices dealt to the XCDs in turn: work-group b (XCD
// b mod 8) takes index ((j / C) 8 + b mod 8) C + j mod C, j = b / 8, over the largest
// multiple of 8 C below nb (the rest keeps its own index).  A chunk keeps its y and z
// neighbours in one L2 while every XCD still gets a share of every part of [0, nb) (the
// batched step: events of unequal cost per item).  A bijection of [0, nb).
template <uint32_t C> GL_HD uint32_t xcd_chunk_remap(uint32_t b, uint32_t nb) {
  const uint32_t whole = nb / (NXCD * C) * (NXCD * C);
  if (b >= whole) return b;
  const uint32_t x = b % NXCD, j = b / NXCD;
  return ((j / C) * NXCD + x) * C + j % C;
}

// Placement of the step's work-groups on the XCDs (work-group b runs on XCD b mod 8,
// each XCD has its own L2).  Two decompositions:
//  * rows: XCD k owns a contiguous range of transverse rows y of every layer and sweeps
//    the layers in order, so the links a block loads as z + 1 neighbours are read again,
//    as z and z - 1, by the blocks that follow on the same XCD; the y halo of the row
//    range crosses XCDs on every layer.
//  * slabs: XCD k owns a contiguous range of layers z, whole, and sweeps them in order;
//    only the two end layers of a slab cross XCDs.
// A block covers BS consecutive sites of one (z, segment) pair, segment = the XCD's row
// range (rows) or the whole layer (slabs); blocks past a segment's end idle.  Slabs are
// the default: with the -z plaquettes taken first (so that a block reads its z - 1
// links while the blocks of that layer read them as their own) the step kernel fetches
// 17% fewer HBM bytes than with rows, at the same speed.
#ifndef GL_ZSLAB
#define GL_ZSLAB 1
#endif
struct ColMap {
  int r0, rem;   // rows (rows) or layers (slabs) per XCD: r0 + (k < rem)
  int bt;        // blocks per (XCD, layer) (rows) or per layer (slabs)
  int slab;      // 1: slab decomposition
};
inline ColMap col_map(const Geom& g, int bs, int slab = GL_ZSLAB) {
  ColMap m;
  m.slab = slab;
  const int n = slab ? g.nz : g.nt;
  m.r0 = n / NXCD;
  m.rem = n % NXCD;
  const int64_t seg = slab ? (int64_t)g.layer : (int64_t)(m.r0 + (m.rem > 0 ? 1 : 0)) * g.nt;
  m.bt = (int)((seg + bs - 1) / bs);
  return m;
}
inline uint32_t col_map_blocks(const Geom& g, const ColMap& m) {
  const int64_t per = m.slab ? (int64_t)(m.r0 + (m.rem > 0 ? 1 : 0)) : (int64_t)g.nz;
  return (uint32_t)(NXCD * per * m.bt);
}
// partial-sum slots per layer: one per block that covers sites of that layer
GL_HD int col_map_slots_per_layer(const ColMap& m) { return m.slab ? m.bt : NXCD * m.bt; }
// layer of block b (may be >= nz or past the XCD's slab for idle blocks) and its slot
GL_HD void col_map_block(const ColMap& m, uint32_t b, int& z, uint32_t& slot) {
  const int k = (int)(b % NXCD);
  const uint32_t j = b / NXCD;
  const uint32_t ch = j % (uint32_t)m.bt;
  if (m.slab) {
    const int zl = (int)(j / (uint32_t)m.bt);
    const int nk = m.r0 + (k < m.rem ? 1 : 0);
    z = zl < nk ? k * m.r0 + (k < m.rem ? k : m.rem) + zl : 0x7fffffff;
    slot = ch;
  } else {
    z = (int)(j / (uint32_t)m.bt);
    slot = (uint32_t)k * m.bt + ch;
  }
}
// site of thread t in block b, or false when the thread has no site
GL_HD bool col_map_site(const Geom& g, const ColMap& m, uint32_t b, uint32_t t, uint32_t bs, Site& x, uint32_t& s) {
  const int k = (int)(b % NXCD);
  const uint32_t j = b / NXCD;
  const uint32_t ch = j % (uint32_t)m.bt;
  const uint32_t local = ch * bs + t;
  int z, y0;
  uint32_t seg;
  if (m.slab) {
    const int zl = (int)(j / (uint32_t)m.bt);
    const int nk = m.r0 + (k < m.rem ? 1 : 0);
    if (zl >= nk) return false;
    z = k * m.r0 + (k < m.rem ? k : m.rem) + zl;
    y0 = 0;
    seg = (uint32_t)g.layer;
  } else {
    z = (int)(j / (uint32_t)m.bt);
    y0 = k * m.r0 + (k < m.rem ? k : m.rem);
    seg = (uint32_t)(m.r0 + (k < m.rem ? 1 : 0)) * (uint32_t)g.nt;
  }
  if (z >= g.nz || local >= seg) return false;
  x.y = y0 + (int)(local / (uint32_t)g.nt);
  x.x = (int)(local % (uint32_t)g.nt);
  x.z = z;
  s = site_index(g, x.x, x.y, x.z);
  return true;
}

// Per-step constants shared by the kernels.
struct StepConst {
  double a[3];       // lattice spacings a_x = a_y = a_T, a_z = a_L
  double dt;
  int hop;           // 1 on a step where every charge advances one cell
  int offA, offB;    // co-moving storage offsets of the two charge populations
  int scheme;        // 0 leapfrog, 1 semi-implicit
};

// Co-moving charge storage: nucleus B (moving +z) keeps the charge that sits at
// physical layer z in slot (z - offB) mod nz; nucleus A (moving -z) in slot
// (z + offA) mod nz.  A hop then only increments the offsets: the parallel
// transport that goes with it rewrites each slot in place.
GL_HD int slotB(int z, int off, int nz) { int r = (z - off) % nz; return r < 0 ? r + nz : r; }
GL_HD int slotA(int z, int off, int nz) { return (z + off) % nz; }

}  // namespace gl
