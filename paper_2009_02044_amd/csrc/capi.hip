// C-ABI of the library (declared in include/glasma.h): context, argument checks,
// the integer charge-hop schedule, host <-> device state transfer and dispatch to
// the templated kernels for (SU(2) | SU(3)) x (double | float).
#include <algorithm>
#include <string>
#include <vector>
#include <cstring>
#include <cstdio>
#include <cmath>
#include <type_traits>
#include "internal.h"
#include "adjoint.h"
#include "../../include/glasma.h"

using namespace gl;

struct glasma_ctx {
  glasma_params p;
  glasma_buffers b;
  hipStream_t stream;
  Geom g;
  int ng, r;          // n_g; reals per link in host arrays (4 or 18)
  int rs;             // reals per link in device storage (4 or 12)
  int64_t step;
  int cur;            // 0: links live in b.U, 1: in b.U_alt
  int offA, offB;     // co-moving charge storage offsets (mod nz)
  int64_t hop_p, hop_q;  // dt / a_L = hop_p / hop_q
  bool ready;
  int last_iters;     // iterations of the last semi-implicit step
  // differentiation form: checkpoints written by glasma_adjoint_forward
  bool adj_ok;
  bool semi_prev;     // semi-implicit: E of the previous step kept (starting guess of the solve)
  int64_t adj_s0;
  int32_t adj_steps, adj_every;
  int adj_off0;
  const void* adj_work;
  int device;         // HIP device current when the context was created
  bool obs_park = true;  // the work buffer holds the observing step's parked projections
  std::string err;
};

static std::string g_err;

static int fail(glasma_ctx* c, int code, const std::string& m) {
  if (c) c->err = m; else g_err = m;
  return code;
}

#define HIPCHK(ctx, call)                                                                     \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) return fail(ctx, GLASMA_E_HIP, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

static bool rational(double r, int64_t* p, int64_t* q) {
  for (int64_t d = 1; d <= 4096; ++d) {
    double n = std::round(r * d);
    if (std::fabs(n / d - r) < 1e-12 && n >= 1) { *p = (int64_t)n; *q = d; return true; }
  }
  return false;
}

// S(s) = floor((s + 1/2) dt/a_L + 1/2) = floor(((2s + 1) p + q) / (2 q)) for s >= -1.
static int64_t hop_count(const glasma_ctx* c, int64_t s) {
  int64_t num = (2 * s + 1) * c->hop_p + c->hop_q;
  int64_t den = 2 * c->hop_q;
  return num >= 0 ? num / den : -((-num + den - 1) / den);
}
static bool is_hop(const glasma_ctx* c, int64_t s) { return hop_count(c, s) > hop_count(c, s - 1); }

static size_t elem(const glasma_params* p) { return p->fp == 64 ? 8 : 4; }
// reals per link in device storage
static int stored_width(const glasma_params* p) { return p->nc == 2 ? 4 : SU3_STORED; }

static int check_params(const glasma_params* p, int64_t* hp, int64_t* hq) {
  if (!p) return fail(nullptr, GLASMA_E_ARG, "params is NULL");
  if (p->nc != 2 && p->nc != 3) return fail(nullptr, GLASMA_E_ARG, "nc must be 2 or 3");
  if (p->nz < 2 || p->nt < 2) return fail(nullptr, GLASMA_E_ARG, "nz and nt must be >= 2");
  if ((int64_t)p->nz * p->nt * p->nt > (int64_t)1 << 31) return fail(nullptr, GLASMA_E_ARG, "lattice too large");
  if (p->fp != 64 && p->fp != 32) return fail(nullptr, GLASMA_E_ARG, "fp must be 64 or 32");
  if (!(p->a_T > 0) || !(p->a_L > 0) || !(p->dt > 0)) return fail(nullptr, GLASMA_E_ARG, "spacings and dt must be > 0");
  if (p->scheme != 0 && p->scheme != 1) return fail(nullptr, GLASMA_E_ARG, "scheme must be 0 or 1");
  if (p->reunit_every < 0) return fail(nullptr, GLASMA_E_ARG, "reunit_every must be >= 0");
  int64_t a, b;
  if (!rational(p->dt / p->a_L, &a, &b) || a > b)
    return fail(nullptr, GLASMA_E_ARG, "dt/a_L must be a rational number in (0, 1] with denominator <= 4096");
  if (hp) *hp = a;
  if (hq) *hq = b;
  return GLASMA_OK;
}

static Geom geom_of(const glasma_params* p) {
  Geom g;
  g.nt = p->nt;
  g.nz = p->nz;
  g.layer = (int64_t)p->nt * p->nt;
  g.V = g.layer * p->nz;
  g.Vp = padded_sites(g.V);
  return g;
}

static size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Work buffer: [general region: initial conditions or observable reductions]
// then, for the semi-implicit scheme, [U(t-dt) | trial links | trial E | f1(U(t), U(t-dt)) | dt j |
// E of the previous step | loops of U(t) alone (marching geometries) | convergence slots].
struct SemiRegion {
  size_t up, ut, et, f2, j, ep, cache, conv, end;  // byte offsets
};
// convergence slots (2 doubles per iteration) of one batch of enqueued iterations
constexpr int SEMI_SLOTS = 64;
static size_t general_bytes(const glasma_params* p) {
  Geom g = geom_of(p);
  int ng = p->nc * p->nc - 1;
  size_t ic = ic_work_doubles(g, ng);
  size_t obs = observe_partial_doubles(g) + 4 * (size_t)g.nz + GLASMA_OBS_NSCALARS;
  size_t loss = adj_loss_partials(g) + 1;
  size_t m = ic > obs ? ic : obs;
  return align256((m > loss ? m : loss) * sizeof(double));
}
static SemiRegion semi_region(const glasma_params* p) {
  Geom g = geom_of(p);
  const size_t e = p->fp == 64 ? 8 : 4;
  const int ng = p->nc * p->nc - 1, r = stored_width(p);
  SemiRegion s;
  s.up = general_bytes(p);
  s.ut = s.up + align256(3 * (size_t)r * g.Vp * e);
  s.et = s.ut + align256(3 * (size_t)r * g.Vp * e);
  s.f2 = s.et + align256(3 * (size_t)ng * g.Vp * e);
  s.j = s.f2 + align256(3 * (size_t)ng * g.Vp * e);
  s.ep = s.j + align256((size_t)ng * g.Vp * e);
  s.cache = s.ep + align256(3 * (size_t)ng * g.Vp * e);
  s.conv = s.cache + (march_geometry(g) ? align256(march_cache_elems(g, p->nc) * e) : 0);
  s.end = s.conv + SEMI_SLOTS * 2 * sizeof(double);
  return s;
}
// Leapfrog: after the general region, the projections parked by the observing step's first
// pass (obs_split_scratch_elems reals of the state's precision).
static size_t work_bytes(const glasma_params* p) {
  if (p->scheme == 1) return semi_region(p).end;
  return general_bytes(p) + align256(obs_split_scratch_elems(geom_of(p), p->nc * p->nc - 1) * elem(p));
}
// The work region of an event of a batch: without the parked projections (the batch steps its
// events itself; an event's own observing step takes the standalone pass instead).
static size_t event_work_bytes(const glasma_params* p) { return general_bytes(p); }

template <class F> static int dispatch(glasma_ctx* c, F&& f) {
  if (c->p.nc == 2 && c->p.fp == 64) return f.template operator()<Su2<double>, double>();
  if (c->p.nc == 3 && c->p.fp == 64) return f.template operator()<Su3<double>, double>();
  if (c->p.nc == 2 && c->p.fp == 32) return f.template operator()<Su2<float>, float>();
  return f.template operator()<Su3<float>, float>();
}

static StepConst step_const(const glasma_ctx* c) {
  StepConst k;
  k.a[0] = c->p.a_T; k.a[1] = c->p.a_T; k.a[2] = c->p.a_L;
  k.dt = c->p.dt;
  k.hop = is_hop(c, c->step) ? 1 : 0;
  k.offA = c->offA;
  k.offB = c->offB;
  k.scheme = c->p.scheme;
  return k;
}

template <typename T> static T* cur_U(glasma_ctx* c) { return (T*)(c->cur ? c->b.U_alt : c->b.U); }
template <typename T> static T* next_U(glasma_ctx* c) { return (T*)(c->cur ? c->b.U : c->b.U_alt); }

// The functions below have C linkage through their declarations in glasma.h.

const char* glasma_version(void) { return "glasma-mi355x 0.1 (gfx950)"; }

const char* glasma_last_error(const glasma_ctx* ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

int glasma_layout(const glasma_params* p, size_t* bytes) {
  int rc = check_params(p, nullptr, nullptr);
  if (rc) return rc;
  if (!bytes) return fail(nullptr, GLASMA_E_ARG, "bytes is NULL");
  Geom g = geom_of(p);
  const size_t e = elem(p);
  const int ng = p->nc * p->nc - 1, r = stored_width(p);
  bytes[0] = 3 * (size_t)r * g.Vp * e;
  bytes[1] = bytes[0];
  bytes[2] = 3 * (size_t)ng * g.Vp * e;
  bytes[3] = (size_t)ng * g.Vp * e;
  bytes[4] = bytes[3];
  bytes[5] = work_bytes(p);
  return GLASMA_OK;
}

int glasma_create(const glasma_params* p, const glasma_buffers* b, void* stream, glasma_ctx** out) {
  int64_t hp, hq;
  int rc = check_params(p, &hp, &hq);
  if (rc) return rc;
  if (!b || !out) return fail(nullptr, GLASMA_E_ARG, "buffers or out is NULL");
  if (!b->U || !b->U_alt || !b->E || !b->rhoA || !b->rhoB || !b->work)
    return fail(nullptr, GLASMA_E_ARG, "a device buffer is NULL");
  if (p->scheme == 1 && (p->max_iter < 1 || !(p->tol > 0)))
    return fail(nullptr, GLASMA_E_ARG, "the semi-implicit scheme needs max_iter >= 1 and tol > 0");
  glasma_ctx* c = new glasma_ctx();
  c->p = *p;
  c->b = *b;
  c->stream = (hipStream_t)stream;
  c->g = geom_of(p);
  c->ng = p->nc * p->nc - 1;
  c->r = p->nc == 2 ? 4 : 18;
  c->rs = stored_width(p);
  c->step = 0;
  c->cur = 0;
  c->offA = c->offB = 0;
  c->hop_p = hp;
  c->hop_q = hq;
  c->ready = false;
  c->last_iters = 0;
  c->adj_ok = false;
  c->device = 0;
  if (hipGetDevice(&c->device) != hipSuccess) c->device = 0;
  *out = c;
  return GLASMA_OK;
}

int glasma_destroy(glasma_ctx* ctx) {
  delete ctx;
  return GLASMA_OK;
}

int glasma_last_iterations(const glasma_ctx* ctx, int32_t* iters) {
  if (!ctx || !iters) return fail(nullptr, GLASMA_E_ARG, "NULL argument");
  *iters = ctx->last_iters;
  return GLASMA_OK;
}

int glasma_get_step(const glasma_ctx* ctx, int64_t* step) {
  if (!ctx || !step) return fail(nullptr, GLASMA_E_ARG, "NULL argument");
  *step = ctx->step;
  return GLASMA_OK;
}

// Host SoA [dir][comp][V] (double) <-> device tiled records (type T), see lattice.h.
// Links: the host array holds host_width reals per link (18 for SU(3)), the device the
// first `width` of them (rows 0 and 1); the third row is rebuilt on load.
template <typename T>
static int upload(glasma_ctx* c, void* dst, const double* src, int ndir, int width, int host_width = 0) {
  const int64_t V = c->g.V, Vp = c->g.Vp;
  if (host_width == 0) host_width = width;
  std::vector<T> tmp((size_t)ndir * width * Vp, T(0));
  for (int d = 0; d < ndir; ++d)
    for (int k = 0; k < width; ++k) {
      const double* sp = src + ((int64_t)d * host_width + k) * V;
      T* dp = tmp.data() + (int64_t)d * width * Vp;
      for (int64_t s = 0; s < V; ++s) dp[rec_elem<T>(s, k, width)] = (T)sp[s];
    }
  HIPCHK(c, hipMemcpyAsync(dst, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return GLASMA_OK;
}

int glasma_init_state(glasma_ctx* c, const double* U, const double* E, const double* rhoA, const double* rhoB,
                      int64_t step0) {
  if (!c || !U || !E || !rhoA || !rhoB) return fail(c, GLASMA_E_ARG, "NULL argument");
  if (step0 < 0) return fail(c, GLASMA_E_ARG, "step0 must be >= 0");
  int rc = dispatch(c, [&]<typename G, typename T>() -> int {
    int r;
    if ((r = upload<T>(c, c->b.U, U, 3, c->rs, c->r))) return r;
    if ((r = upload<T>(c, c->b.E, E, 3, c->ng))) return r;
    if ((r = upload<T>(c, c->b.rhoA, rhoA, 1, c->ng))) return r;
    if ((r = upload<T>(c, c->b.rhoB, rhoB, 1, c->ng))) return r;
    return GLASMA_OK;
  });
  if (rc) return rc;
  c->cur = 0;
  c->offA = c->offB = 0;
  c->step = step0;
  c->ready = true;
  c->semi_prev = false;
  c->adj_ok = false;
  return GLASMA_OK;
}

int glasma_init_mv_sheets(glasma_ctx* c, const glasma_mv* mv, int32_t ns, const double* rhoT_A,
                          const double* rhoT_B) {
  if (!c || !mv || !rhoT_A || !rhoT_B) return fail(c, GLASMA_E_ARG, "NULL argument");
  if (!(mv->m_ir > 0) || !(mv->sigma > 0)) return fail(c, GLASMA_E_ARG, "m_ir and sigma must be > 0");
  if (ns < 1) return fail(c, GLASMA_E_ARG, "ns must be >= 1");
  const size_t m = (size_t)c->ng * c->g.layer;
  // the fields of several sheets are held in the second link buffer, free until the first step
  const size_t ubytes = 3 * (size_t)c->rs * c->g.Vp * (c->p.fp == 64 ? 8 : 4);
  if (ns > 1 && (size_t)ns * 2 * m * sizeof(double) > ubytes)
    return fail(c, GLASMA_E_ARG, "too many sheets for this lattice (ns * 2 * n_g * nt^2 doubles must fit the "
                                 "second link buffer)");
  double* work = (double*)c->b.work;
  double* phi = ns == 1 ? work + 2 * m : (double*)c->b.U_alt;
  McvConst k{mv->m_ir, mv->uv_cut, mv->sigma, mv->zA, mv->zB};
  c->adj_ok = false;
  c->step = 0;
  c->cur = 0;
  c->offA = c->offB = 0;
  StepConst sc = step_const(c);
  for (int32_t q = 0; q < ns; ++q) {
    HIPCHK(c, hipMemcpyAsync(work, rhoT_A + q * m, m * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(work + m, rhoT_B + q * m, m * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    launch_ic_phi(work, phi + (size_t)q * 2 * m, c->ng, c->g, sc, k, c->stream);
  }
  dispatch(c, [&]<typename G, typename T>() -> int {
    launch_ic_fields<G, T>(phi, ns, (T*)c->b.U, (T*)c->b.E, (T*)c->b.rhoA, (T*)c->b.rhoB, c->g, sc, k, c->stream);
    if (c->p.scheme == 1) {
      // charges that make the conserved combination D.(E + dt f1(U(t0), U(t0 - dt))) - rho vanish
      const SemiRegion r = semi_region(&c->p);
      char* w = (char*)c->b.work;
      launch_semi_begin<G, T>((T*)c->b.U, (T*)c->b.E, (const T*)nullptr, (const T*)nullptr, (T*)(w + r.up),
                              (T*)(w + r.ut), (T*)(w + r.et), c->g, sc,
                              c->stream);
      launch_semi_f1<G, T>((T*)c->b.U, (T*)(w + r.up), (T*)(w + r.f2), c->g, sc, c->stream);
      launch_gauss_charges<G, T>((T*)c->b.U, (T*)c->b.E, (T*)(w + r.f2), c->p.dt, (T*)c->b.rhoA,
                                 (T*)c->b.rhoB, c->g, sc, c->stream);
    }
    return 0;
  });
  HIPCHK(c, hipGetLastError());
  c->ready = true;
  c->semi_prev = false;
  return GLASMA_OK;
}

int glasma_init_mv(glasma_ctx* c, const glasma_mv* mv, const double* rhoT_A, const double* rhoT_B) {
  return glasma_init_mv_sheets(c, mv, 1, rhoT_A, rhoT_B);
}

// ---- boost-invariant tau = 0+ fields of two nuclei ------------------------------

int glasma_bi_work_bytes(const glasma_params* p, size_t* bytes) {
  int rc = check_params(p, nullptr, nullptr);
  if (rc) return rc;
  if (!bytes) return fail(nullptr, GLASMA_E_ARG, "bytes is NULL");
  const Geom g = geom_of(p);
  *bytes = bi_work_doubles(g, p->nc * p->nc - 1, p->nc == 3 ? 18 : 4) * sizeof(double);
  return GLASMA_OK;
}

int glasma_bi_fields(const glasma_params* p, const glasma_mv* mv, int32_t ns, const double* rhoT_A,
                     const double* rhoT_B, void* work, double* Ez, double* Bz, double* out3, void* stream) {
  int rc = check_params(p, nullptr, nullptr);
  if (rc) return rc;
  if (!mv || !rhoT_A || !rhoT_B || !work || !Ez || !Bz || !out3) return fail(nullptr, GLASMA_E_ARG, "NULL argument");
  if (!(mv->m_ir > 0)) return fail(nullptr, GLASMA_E_ARG, "m_ir must be > 0");
  if (ns < 1) return fail(nullptr, GLASMA_E_ARG, "ns must be >= 1");
  const Geom g = geom_of(p);
  const int ng = p->nc * p->nc - 1;
  const size_t m = (size_t)ng * g.layer;
  hipStream_t st = (hipStream_t)stream;
  double* w = (double*)work;
  double* phi = w + 2 * m;
  double* links = w + ic_work_doubles(g, ng);
  double* partial = links + 2 * (size_t)g.layer * (p->nc == 3 ? 18 : 4);
  StepConst sc{};
  sc.a[0] = sc.a[1] = p->a_T;
  sc.a[2] = p->a_L;
  sc.dt = p->dt;
  McvConst k{mv->m_ir, mv->uv_cut, mv->sigma, mv->zA, mv->zB};
  for (int32_t q = 0; q < ns; ++q) {
    HIPCHK(nullptr, hipMemcpyAsync(w, rhoT_A + q * m, m * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(nullptr, hipMemcpyAsync(w + m, rhoT_B + q * m, m * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(nullptr, hipStreamSynchronize(st));
    launch_ic_phi(w, phi, ng, g, sc, k, st);
    if (p->nc == 3) launch_bi_sheet<3>(phi, links, g, q == 0, st);
    else launch_bi_sheet<2>(phi, links, g, q == 0, st);
  }
  if (p->nc == 3) launch_bi_fields<3>(links, partial, g, p->a_T, Ez, Bz, out3, st);
  else launch_bi_fields<2>(links, partial, g, p->a_T, Ez, Bz, out3, st);
  HIPCHK(nullptr, hipGetLastError());
  return GLASMA_OK;
}

// Semi-implicit solve of the step from the current state: the current of the hop (the
// charges stay where they are), U(t - dt) and f1(U(t), U(t - dt)) once, then fixed-point
// iterations on E(t + dt/2) until max|dE| <= tol max|E|.  Iterations are enqueued in batches
// (the first as long as the last step needed, plus one); each writes its convergence slot
// and does nothing once the slot before it has converged, so the host reads the slots once
// per batch.  On success the converged E(t + dt/2) is in the work region's trial E and
// *links points at the new links (next_U or the trial-link buffer).  Nothing of the state
// (links, E, charges, step) is changed, so an error leaves the state as it was.
static int semi_solve(glasma_ctx* c, const StepConst& sc, void** links) {
  const SemiRegion r = semi_region(&c->p);
  char* w = (char*)c->b.work;
  double* conv = (double*)(w + r.conv);
  return dispatch(c, [&]<typename G, typename T>() -> int {
    T* Uc = cur_U<T>(c);
    T* Up = (T*)(w + r.up);
    T* Et = (T*)(w + r.et);
    T* F2 = (T*)(w + r.f2);
    T* J = (T*)(w + r.j);
    T* Ep = (T*)(w + r.ep);
    // the current first: it enters the starting guess
    if (sc.hop) launch_semi_hop<G, T>(Uc, (T*)c->b.rhoA, (T*)c->b.rhoB, J, false, c->g, sc, c->stream);
    T* buf[2] = {next_U<T>(c), (T*)(w + r.ut)};   // iteration k reads buf[k & 1], writes buf[(k + 1) & 1]
    launch_semi_begin<G, T>(Uc, (T*)c->b.E, c->semi_prev ? Ep : nullptr, sc.hop ? J : nullptr, Up, buf[0], Et, c->g,
                            sc, c->stream);
    T* cache = march_geometry(c->g) ? (T*)(w + r.cache) : nullptr;
    launch_semi_f1<G, T>(Uc, Up, F2, c->g, sc, c->stream, cache);
    launch_semi_base<G, T>((const T*)c->b.E, F2, sc.hop ? J : nullptr, c->g, c->p.dt, c->stream);
    double h[2 * SEMI_SLOTS];
    int done = 0, at = -1;
    while (done < c->p.max_iter && at < 0) {
      int nb = done == 0 ? std::max(c->last_iters + 1, 3) : 4;
      nb = std::min(std::min(nb, SEMI_SLOTS), c->p.max_iter - done);
      launch_zero(conv, 2 * nb, c->stream);
      for (int k = 0; k < nb; ++k) {
        const int it = done + k;
        launch_semi_iter<G, T>(Uc, buf[it & 1], F2, Et, buf[(it + 1) & 1], conv + 2 * k,
                               k ? conv + 2 * (k - 1) : nullptr, c->p.tol, c->g, sc, c->stream, cache);
      }
      HIPCHK(c, hipGetLastError());
      HIPCHK(c, hipMemcpyAsync(h, conv, 2 * nb * sizeof(double), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      for (int k = 0; k < nb; ++k) {
        const double d = h[2 * k], e = h[2 * k + 1];
        if (!std::isfinite(d) || !std::isfinite(e)) {
          c->last_iters = done + k + 1;
          return fail(c, GLASMA_E_NONFINITE, "non-finite field in the semi-implicit solve");
        }
        if (d <= c->p.tol * (e > 0 ? e : 1e-300)) { at = done + k; break; }
      }
      done += nb;
    }
    if (at < 0) {
      c->last_iters = done;
      return fail(c, GLASMA_E_NOCONV, "semi-implicit iteration reached max_iter");
    }
    c->last_iters = at + 1;
    *links = buf[(at + 1) & 1];
    return GLASMA_OK;
  });
}

// Accept a converged solve: new links into next_U, the reference of the next step's
// starting guess, E(t + dt/2) into E, and the hop of the charges (with U(t)).
static int semi_commit(glasma_ctx* c, const StepConst& sc, void* links) {
  const SemiRegion r = semi_region(&c->p);
  char* w = (char*)c->b.work;
  dispatch(c, [&]<typename G, typename T>() -> int {
    T* Un = next_U<T>(c);
    T* J = (T*)(w + r.j);
    const int64_t nl = 3 * (int64_t)c->rs * c->g.Vp, ne = 3 * (int64_t)c->ng * c->g.Vp;
    if ((T*)links != Un) launch_copy<G, T>((const T*)links, Un, nl, c->stream);
    launch_semi_keep<G, T>((T*)c->b.E, sc.hop ? J : nullptr, (T*)(w + r.ep), c->g, c->stream);
    launch_copy<G, T>((const T*)(w + r.et), (T*)c->b.E, ne, c->stream);
    if (sc.hop) launch_semi_hop<G, T>(cur_U<T>(c), (T*)c->b.rhoA, (T*)c->b.rhoB, J, true, c->g, sc, c->stream);
    return 0;
  });
  c->semi_prev = true;
  HIPCHK(c, hipGetLastError());
  return GLASMA_OK;
}

// Observables of the current state for the semi-implicit scheme, with E(t + dt/2) from the
// converged solve of the step that follows (its trial E in the work region).
static int semi_observe_solved(glasma_ctx* c, const StepConst& sc, double* d_obs) {
  const SemiRegion r = semi_region(&c->p);
  char* w = (char*)c->b.work;
  double* partial = (double*)c->b.work;
  dispatch(c, [&]<typename G, typename T>() -> int {
    launch_observe<G, T>(cur_U<T>(c), (T*)c->b.E, (T*)c->b.rhoA, (T*)c->b.rhoB, (const T*)(w + r.et), c->g, sc,
                         partial, d_obs, c->stream);
    return 0;
  });
  HIPCHK(c, hipGetLastError());
  return GLASMA_OK;
}

static int advance(glasma_ctx* c, int32_t n);
static int observe_leapfrog(glasma_ctx* c, const StepConst& sc, double* partial, double* d_out);

int glasma_step(glasma_ctx* c, int32_t n) {
  if (!c) return fail(nullptr, GLASMA_E_ARG, "NULL context");
  if (n < 0) return fail(c, GLASMA_E_ARG, "n must be >= 0");
  if (!c->ready) return fail(c, GLASMA_E_STATE, "no state: call glasma_init_state or glasma_init_mv first");
  c->adj_ok = false;
  return advance(c, n);
}

// Which observing step the FP64 leapfrog takes where the step kernel can gather the energy
// slots itself (nt a multiple of 64): 1 that fused step, 0 the passes around a plain step.
#ifndef GL_OBS_FUSED64
#define GL_OBS_FUSED64 1
#endif

// One step; with d_obs (the observing step) it also writes to d_obs the observables of the
// state it starts from.  Leapfrog: a pass over that state (Gauss residual, magnetic and
// E(t - dt/2) parts, parked plaquette projections), the plain step, and a pass adding the
// E(t + dt/2) parts; or, for FP64 with nt a multiple of 64, the Gauss residual kernel and a
// step kernel that adds the energy slots.  Semi-implicit scheme: the observables pass runs
// between the converged solve and its commit, with E(t + dt/2) from the solve.
static int one_step(glasma_ctx* c, double* d_obs) {
  StepConst sc = step_const(c);
  // reunitarisation after this step: inside the plain leapfrog step, else a pass after it
  const bool ru = c->p.reunit_every > 0 && (c->step + 1) % c->p.reunit_every == 0;
  bool ru_done = false;
  if (c->p.scheme == 1) {
    void* links = nullptr;
    int rc = semi_solve(c, sc, &links);
    if (rc) return rc;
    if (d_obs && (rc = semi_observe_solved(c, sc, d_obs))) return rc;
    if ((rc = semi_commit(c, sc, links))) return rc;
  } else if (d_obs && !(GL_OBS_FUSED64 && c->p.fp == 64 && fused_observe_geometry(c->g)) && !c->obs_park) {
    // no room for the parked projections (an event of a batch): the standalone pass, then the step
    int rc = observe_leapfrog(c, sc, (double*)c->b.work, d_obs);
    if (rc) return rc;
    dispatch(c, [&]<typename G, typename T>() -> int {
      launch_leapfrog<G, T>(cur_U<T>(c), next_U<T>(c), (T*)c->b.E, (T*)c->b.rhoA, (T*)c->b.rhoB, c->g, sc,
                            ru, c->stream);
      return 0;
    });
    ru_done = ru;
  } else if (d_obs && !(GL_OBS_FUSED64 && c->p.fp == 64 && fused_observe_geometry(c->g))) {
    double* partial = (double*)c->b.work;
    dispatch(c, [&]<typename G, typename T>() -> int {
      T* Q = (T*)((char*)c->b.work + general_bytes(&c->p));
      launch_obs_pre<G, T>(cur_U<T>(c), (T*)c->b.E, (T*)c->b.rhoA, (T*)c->b.rhoB, c->g, sc, Q, partial, c->stream);
      launch_leapfrog<G, T>(cur_U<T>(c), next_U<T>(c), (T*)c->b.E, (T*)c->b.rhoA, (T*)c->b.rhoB, c->g, sc, ru,
                            c->stream);
      launch_obs_post<G, T>((T*)c->b.E, Q, c->g, sc, partial, d_obs, c->stream);
      return 0;
    });
    ru_done = ru;
  } else if (d_obs) {
    double* partial = (double*)c->b.work;
    dispatch(c, [&]<typename G, typename T>() -> int {
      if constexpr (std::is_same_v<T, double>) {
        launch_obs_gauss<G, T>(cur_U<T>(c), (T*)c->b.E, (T*)c->b.rhoA, (T*)c->b.rhoB, c->g, sc, partial,
                               c->stream);
        launch_leapfrog_observe<G, T>(cur_U<T>(c), next_U<T>(c), (T*)c->b.E, (T*)c->b.rhoA, (T*)c->b.rhoB, c->g,
                                      sc, partial, c->stream);
      }
      return 0;
    });
    launch_observe_finish(partial, fused_observe_blocks_per_layer(c->g), c->g, sc, d_obs, c->stream);
  } else {
    dispatch(c, [&]<typename G, typename T>() -> int {
      launch_leapfrog<G, T>(cur_U<T>(c), next_U<T>(c), (T*)c->b.E, (T*)c->b.rhoA, (T*)c->b.rhoB, c->g, sc,
                            ru, c->stream);
      return 0;
    });
    ru_done = ru;
  }
  c->cur ^= 1;
  if (sc.hop) {
    c->offA = (c->offA + 1) % c->g.nz;
    c->offB = (c->offB + 1) % c->g.nz;
  }
  c->step += 1;
  if (ru && !ru_done) {
    dispatch(c, [&]<typename G, typename T>() -> int {
      launch_reunit<G, T>(cur_U<T>(c), c->g, c->stream);
      return 0;
    });
  }
  HIPCHK(c, hipGetLastError());
  return GLASMA_OK;
}

static int advance(glasma_ctx* c, int32_t n) {
  for (int32_t k = 0; k < n; ++k) {
    int rc = one_step(c, nullptr);
    if (rc) return rc;
  }
  return GLASMA_OK;
}

int glasma_step_observe(glasma_ctx* c, int32_t n, double* d_out) {
  if (!c || !d_out) return fail(c, GLASMA_E_ARG, "NULL argument");
  if (n < 1) return fail(c, GLASMA_E_ARG, "n must be >= 1");
  if (!c->ready) return fail(c, GLASMA_E_STATE, "no state: call glasma_init_state or glasma_init_mv first");
  c->adj_ok = false;
  int rc = advance(c, n - 1);
  if (rc) return rc;
  return one_step(c, d_out);
}

int glasma_reunitarize(glasma_ctx* c) {
  if (!c) return fail(nullptr, GLASMA_E_ARG, "NULL context");
  if (!c->ready) return fail(c, GLASMA_E_STATE, "no state");
  c->adj_ok = false;
  dispatch(c, [&]<typename G, typename T>() -> int {
    launch_reunit<G, T>(cur_U<T>(c), c->g, c->stream);
    return 0;
  });
  HIPCHK(c, hipGetLastError());
  return GLASMA_OK;
}

int glasma_deposit_current(glasma_ctx* c, void* j_out) {
  if (!c || !j_out) return fail(c, GLASMA_E_ARG, "NULL argument");
  if (!c->ready) return fail(c, GLASMA_E_STATE, "no state");
  StepConst sc = step_const(c);
  dispatch(c, [&]<typename G, typename T>() -> int {
    launch_current<G, T>(cur_U<T>(c), (T*)c->b.rhoA, (T*)c->b.rhoB, c->g, sc, (T*)j_out, c->stream);
    return 0;
  });
  HIPCHK(c, hipGetLastError());
  return GLASMA_OK;
}

// Observables of the leapfrog state with the per-block partial sums in `partial`
// (observe_partial_doubles doubles of device memory).
static int observe_leapfrog(glasma_ctx* c, const StepConst& sc, double* partial, double* d_out) {
  dispatch(c, [&]<typename G, typename T>() -> int {
    launch_observe<G, T>(cur_U<T>(c), (T*)c->b.E, (T*)c->b.rhoA, (T*)c->b.rhoB, (const T*)nullptr, c->g, sc, partial,
                         d_out, c->stream);
    return 0;
  });
  HIPCHK(c, hipGetLastError());
  return GLASMA_OK;
}

int glasma_observe(glasma_ctx* c, double* d_out) {
  if (!c || !d_out) return fail(c, GLASMA_E_ARG, "NULL argument");
  if (!c->ready) return fail(c, GLASMA_E_STATE, "no state");
  StepConst sc = step_const(c);
  if (c->p.scheme == 1) {
    // E(t + dt/2) needs the solve of the next step: solve it, observe, and discard it
    const int iters = c->last_iters;
    void* links = nullptr;
    int rc = semi_solve(c, sc, &links);
    c->last_iters = iters;
    if (rc) return rc;
    return semi_observe_solved(c, sc, d_out);
  }
  return observe_leapfrog(c, sc, (double*)c->b.work, d_out);
}

int glasma_observe_noalloc(glasma_ctx* c, double* d_out) {
  if (!c || !d_out) return fail(c, GLASMA_E_ARG, "NULL argument");
  if (!c->ready) return fail(c, GLASMA_E_STATE, "no state");
  if (c->p.scheme != 0)
    return fail(c, GLASMA_E_ARG, "glasma_observe_noalloc covers the leapfrog scheme (the semi-implicit observables "
                                 "need the solve of the next step)");
  double* scratch = nullptr;
  size_t cap = 0;
  HIPCHK(c, observe_static_scratch(c->device, &scratch, &cap));
  if (observe_partial_doubles(c->g) > cap)
    return fail(c, GLASMA_E_ARG, "lattice too large for glasma_observe_noalloc: its partial sums need " +
                                     std::to_string(observe_partial_doubles(c->g)) + " doubles, the static scratch "
                                     "holds " + std::to_string(cap) + " (use glasma_observe)");
  return observe_leapfrog(c, step_const(c), scratch, d_out);
}

int glasma_rest_frame(glasma_ctx* c, const double* d_obs, double* d_out) {
  if (!c || !d_obs || !d_out) return fail(c, GLASMA_E_ARG, "NULL argument");
  launch_rest_frame(d_obs, c->g.nz, d_out, c->stream);
  HIPCHK(c, hipGetLastError());
  return GLASMA_OK;
}

int glasma_observables(glasma_ctx* c, double* tmunu_z, double* gauss_rel, double* gauss_max, double* energy,
                       double* unitarity_max) {
  if (!c) return fail(nullptr, GLASMA_E_ARG, "NULL context");
  const size_t nout = 4 * (size_t)c->g.nz + GLASMA_OBS_NSCALARS;
  double* d_out = (double*)c->b.work + observe_partial_doubles(c->g);
  int rc = glasma_observe(c, d_out);
  if (rc) return rc;
  std::vector<double> h(nout);
  HIPCHK(c, hipMemcpyAsync(h.data(), d_out, nout * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const double* s = h.data() + 4 * c->g.nz;
  if (tmunu_z) std::memcpy(tmunu_z, h.data(), 4 * c->g.nz * sizeof(double));
  if (gauss_rel) *gauss_rel = s[GLASMA_OBS_GAUSS_REL];
  if (gauss_max) *gauss_max = s[GLASMA_OBS_GAUSS_MAX];
  if (energy) *energy = s[GLASMA_OBS_ENERGY];
  if (unitarity_max) *unitarity_max = s[GLASMA_OBS_UNITARITY];
  if (s[GLASMA_OBS_NONFINITE] > 0) return fail(c, GLASMA_E_NONFINITE, "non-finite values in the fields");
  return GLASMA_OK;
}

// zsrc(z) gives the stored layer that holds physical layer z (co-moving charges).
// Links (host_width 18 > width 12): the third row of each SU(3) matrix is rebuilt as
// conj(row 0 x row 1), as the kernels do on load.
template <typename T, typename F>
static int download(glasma_ctx* c, double* dst, const void* src, int ndir, int width, F zsrc, int host_width = 0) {
  const int64_t V = c->g.V, Vp = c->g.Vp, layer = c->g.layer;
  if (host_width == 0) host_width = width;
  std::vector<T> tmp((size_t)ndir * width * Vp);
  HIPCHK(c, hipMemcpyAsync(tmp.data(), src, tmp.size() * sizeof(T), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int d = 0; d < ndir; ++d) {
    for (int k = 0; k < width; ++k) {
      double* dp = dst + ((int64_t)d * host_width + k) * V;
      const T* sp = tmp.data() + (int64_t)d * width * Vp;
      for (int z = 0; z < c->g.nz; ++z) {
        const int64_t zs = zsrc(z);
        for (int64_t t = 0; t < layer; ++t) dp[z * layer + t] = (double)sp[rec_elem<T>(zs * layer + t, k, width)];
      }
    }
    if (host_width == 18 && width == SU3_STORED) {
      double* base = dst + (int64_t)d * host_width * V;
      auto at = [&](int r, int k, int im) { return base[(2 * (3 * r + k) + im) * V]; };
      for (int64_t s = 0; s < V; ++s, ++base) {
        for (int k = 0; k < 3; ++k) {
          const int a = (k + 1) % 3, b = (k + 2) % 3;
          const double cr = at(0, a, 0) * at(1, b, 0) - at(0, a, 1) * at(1, b, 1) - (at(0, b, 0) * at(1, a, 0) - at(0, b, 1) * at(1, a, 1));
          const double ci = at(0, a, 0) * at(1, b, 1) + at(0, a, 1) * at(1, b, 0) - (at(0, b, 0) * at(1, a, 1) + at(0, b, 1) * at(1, a, 0));
          base[(2 * (6 + k)) * V] = cr;
          base[(2 * (6 + k) + 1) * V] = -ci;
        }
      }
    }
  }
  return GLASMA_OK;
}

int glasma_get_state(glasma_ctx* c, double* U, double* E, double* rhoA, double* rhoB, int64_t* step) {
  if (!c) return fail(nullptr, GLASMA_E_ARG, "NULL context");
  if (!c->ready) return fail(c, GLASMA_E_STATE, "no state");
  const int nz = c->g.nz;
  int rc = dispatch(c, [&]<typename G, typename T>() -> int {
    int r;
    auto same = [](int z) { return z; };
    const int oA = c->offA, oB = c->offB;
    if (U && (r = download<T>(c, U, cur_U<T>(c), 3, c->rs, same, c->r))) return r;
    if (E && (r = download<T>(c, E, c->b.E, 3, c->ng, same))) return r;
    if (rhoA && (r = download<T>(c, rhoA, c->b.rhoA, 1, c->ng, [&](int z) { return slotA(z, oA, nz); }))) return r;
    if (rhoB && (r = download<T>(c, rhoB, c->b.rhoB, 1, c->ng, [&](int z) { return slotB(z, oB, nz); }))) return r;
    return GLASMA_OK;
  });
  if (rc) return rc;
  if (step) *step = c->step;
  return GLASMA_OK;
}

// ---- host evaluation of the group kernels -----------------------------------
template <typename G>
static void host_op(int op, int64_t n, const double* in, double* out) {
  using T = typename G::Real;
  constexpr int NG = G::NG, R = G::R;
  auto rd_link = [](const double* p) {
    typename G::Link l;
    T* q = reinterpret_cast<T*>(&l);
    if constexpr (R == 4) { for (int k = 0; k < 4; ++k) q[k] = (T)p[k]; }
    else {
      for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) { l.re[r][k] = (T)p[2 * (3 * r + k)]; l.im[r][k] = (T)p[2 * (3 * r + k) + 1]; }
    }
    return l;
  };
  auto wr_link = [](const typename G::Link& l, double* p) {
    const T* q = reinterpret_cast<const T*>(&l);
    if constexpr (R == 4) { for (int k = 0; k < 4; ++k) p[k] = q[k]; }
    else {
      for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) { p[2 * (3 * r + k)] = l.re[r][k]; p[2 * (3 * r + k) + 1] = l.im[r][k]; }
    }
  };
  auto rd_alg = [](const double* p) { typename G::Alg a; for (int k = 0; k < NG; ++k) a.c[k] = (T)p[k]; return a; };
  auto wr_alg = [](const typename G::Alg& a, double* p) { for (int k = 0; k < NG; ++k) p[k] = a.c[k]; };
  for (int64_t it = 0; it < n; ++it) {
    switch (op) {
      case 0: wr_link(G::expi(rd_alg(in + 1), (T)in[0]), out); in += NG + 1; out += R; break;
      case 1: wr_alg(G::logi(rd_link(in)), out); in += R; out += NG; break;
      case 2: wr_alg(G::proj(rd_link(in)), out); in += R; out += NG; break;
      case 3: wr_alg(G::transport(rd_link(in), rd_alg(in + R)), out); in += R + NG; out += NG; break;
      case 4: wr_link(G::reunit(rd_link(in)), out); in += R; out += R; break;
      case 5: out[0] = G::unit_violation(rd_link(in)); in += R; out += 1; break;
      case 6: wr_link(G::mul(rd_link(in), rd_link(in + R)), out); in += 2 * R; out += R; break;
      case 7: {
        // transpose of the exponential's derivative, always in double (the adjoint's arithmetic)
        using Gd = typename GroupOf<G::NC, double>::type;
        typename Gd::Alg e, l;
        for (int k = 0; k < NG; ++k) { e.c[k] = in[1 + k]; l.c[k] = in[1 + NG + k]; }
        const typename Gd::Alg r = dexp_transpose<Gd>(e, in[0], l);
        for (int k = 0; k < NG; ++k) out[k] = r.c[k];
        in += 1 + 2 * NG;
        out += NG;
        break;
      }
    }
  }
}

int glasma_host_group_op(int32_t nc, int32_t fp, int32_t op, int64_t n, const double* in, double* out) {
  if ((nc != 2 && nc != 3) || (fp != 64 && fp != 32) || op < 0 || op > 7 || n < 0 || (n > 0 && (!in || !out)))
    return fail(nullptr, GLASMA_E_ARG, "bad arguments to glasma_host_group_op");
  if (nc == 2 && fp == 64) host_op<Su2<double>>(op, n, in, out);
  else if (nc == 3 && fp == 64) host_op<Su3<double>>(op, n, in, out);
  else if (nc == 2) host_op<Su2<float>>(op, n, in, out);
  else host_op<Su3<float>>(op, n, in, out);
  return GLASMA_OK;
}


// ============================================================================
// Batched form: many events of different lattice sizes advanced together by one
// launch per step over (event, block of sites) work items, replayed from a
// captured HIP graph.  Each event is a full context over its own slice of the pool.
// ============================================================================
struct glasma_batch {
  glasma_params p;                 // common parameters (nz, nt unused)
  std::vector<glasma_ctx*> ev;
  std::vector<size_t> ev_off;      // byte offset of each event's buffers in the pool
  char* pool;
  hipStream_t stream;
  EventDesc* d_ev;                 // device event table
  uint32_t* d_item_event;          // device item -> event map
  int64_t* d_ctr;                  // device step counter
  uint32_t items_for_bs[257];      // item count for each sites-per-item value (cached lazily)
  int bs, grid;                    // chosen sites per item and persistent grid (0 = one per item)
  hipGraph_t graph;
  hipGraphExec_t exec;
  int graph_steps, graph_bs, graph_grid;
  // event averages: every event's observables buffer, the averaging table, N_z classes
  double* d_obs;
  std::vector<int64_t> obs_off;    // doubles from d_obs to each event's buffer
  BatchObsEvent* d_avg_ev;
  int* d_cls;                      // [n] class N_z | [n + 1] class offsets | [n] class counts
  std::vector<int> cls_nz, cls_off, cls_count;
  std::string err;
  std::string tune_report;
};

static int bfail(glasma_batch* b, int code, const std::string& m) {
  if (b) b->err = m; else g_err = m;
  return code;
}

#define BHIPCHK(b, call)                                                                                  \
  do {                                                                                                    \
    hipError_t e_ = (call);                                                                               \
    if (e_ != hipSuccess) return bfail(b, GLASMA_E_HIP, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

static glasma_params event_params(const glasma_params* common, int32_t nz, int32_t nt) {
  glasma_params q = *common;
  q.nz = nz;
  q.nt = nt;
  q.scheme = 0;
  return q;
}

// pool layout: per event [U | U_alt | E | rhoA | rhoB | work], then the event table,
// the item map for the smallest work item (64 sites), the step counter, every event's
// observables buffer (4 nz + GLASMA_OBS_NSCALARS doubles) and the averaging tables
struct BatchLayout {
  std::vector<size_t> ev;          // byte offset of each event's buffers
  std::vector<int64_t> obs;        // doubles from the observables region to each event's buffer
  size_t table, items, ctr, obs_region, avg_ev, cls, total;
};
static int batch_sizes(const glasma_params* common, int32_t n, const int32_t* nz, const int32_t* nt,
                       BatchLayout* L) {
  if (!common || n < 1 || !nz || !nt) return fail(nullptr, GLASMA_E_ARG, "bad batch arguments");
  if (common->scheme != 0) return fail(nullptr, GLASMA_E_ARG, "the batched form runs the leapfrog scheme");
  size_t off = 0;
  uint64_t items64 = 0;
  int64_t nobs = 0;
  for (int32_t e = 0; e < n; ++e) {
    glasma_params q = event_params(common, nz[e], nt[e]);
    size_t b[6];
    int rc = glasma_layout(&q, b);
    if (rc) return rc;
    b[5] = event_work_bytes(&q);
    L->ev.push_back(off);
    for (int k = 0; k < 6; ++k) off += align256(b[k]);
    items64 += (uint64_t)(geom_of(&q).V + 63) / 64;
    L->obs.push_back(nobs);
    nobs += 4 * (int64_t)nz[e] + GLASMA_OBS_NSCALARS;
  }
  L->table = off;
  off += align256((size_t)n * sizeof(EventDesc));
  L->items = off;
  off += align256((size_t)items64 * sizeof(uint32_t));
  L->ctr = off;
  off += 256;
  L->obs_region = off;
  off += align256((size_t)nobs * sizeof(double));
  L->avg_ev = off;
  off += align256((size_t)n * sizeof(BatchObsEvent));
  L->cls = off;
  off += align256((size_t)(3 * n + 1) * sizeof(int));
  L->total = off;
  return GLASMA_OK;
}

int glasma_batch_layout(const glasma_params* common, int32_t n_events, const int32_t* nz, const int32_t* nt,
                        size_t* pool_bytes) {
  BatchLayout L;
  int rc = batch_sizes(common, n_events, nz, nt, &L);
  if (rc) return rc;
  if (!pool_bytes) return fail(nullptr, GLASMA_E_ARG, "pool_bytes is NULL");
  *pool_bytes = L.total;
  return GLASMA_OK;
}

int glasma_batch_create(const glasma_params* common, int32_t n_events, const int32_t* nz, const int32_t* nt,
                        void* pool, void* stream, glasma_batch** out) {
  BatchLayout L;
  int rc = batch_sizes(common, n_events, nz, nt, &L);
  if (rc) return rc;
  const std::vector<size_t>& offs = L.ev;
  const size_t toff = L.table, ioff = L.items, coff = L.ctr;
  if (!pool || !out) return fail(nullptr, GLASMA_E_ARG, "pool or out is NULL");
  glasma_batch* b = new glasma_batch();
  b->p = *common;
  b->pool = (char*)pool;
  b->stream = (hipStream_t)stream;
  b->ev_off = offs;
  for (int32_t e = 0; e < n_events; ++e) {
    glasma_params q = event_params(common, nz[e], nt[e]);
    size_t sz[6];
    glasma_layout(&q, sz);
    sz[5] = event_work_bytes(&q);
    char* base = b->pool + offs[e];
    glasma_buffers bf;
    void** slots[6] = {&bf.U, &bf.U_alt, &bf.E, &bf.rhoA, &bf.rhoB, &bf.work};
    size_t o = 0;
    for (int k = 0; k < 6; ++k) { *slots[k] = base + o; o += align256(sz[k]); }
    glasma_ctx* c = nullptr;
    rc = glasma_create(&q, &bf, stream, &c);
    if (rc) {
      for (auto* x : b->ev) glasma_destroy(x);
      delete b;
      return rc;
    }
    c->obs_park = false;
    b->ev.push_back(c);
  }
  b->d_ev = (EventDesc*)(b->pool + toff);
  b->d_item_event = (uint32_t*)(b->pool + ioff);
  b->d_ctr = (int64_t*)(b->pool + coff);
  b->bs = 256;
  b->grid = 0;
  b->graph = nullptr;
  b->exec = nullptr;
  b->graph_steps = b->graph_bs = b->graph_grid = 0;
  // N_z classes (ascending) and the averaging tables
  b->d_obs = (double*)(b->pool + L.obs_region);
  b->obs_off = L.obs;
  b->d_avg_ev = (BatchObsEvent*)(b->pool + L.avg_ev);
  b->d_cls = (int*)(b->pool + L.cls);
  std::vector<int> nzs(nz, nz + n_events);
  std::sort(nzs.begin(), nzs.end());
  nzs.erase(std::unique(nzs.begin(), nzs.end()), nzs.end());
  b->cls_nz = nzs;
  b->cls_count.assign(nzs.size(), 0);
  std::vector<BatchObsEvent> tab(n_events);
  for (int32_t e = 0; e < n_events; ++e) {
    const int k = (int)(std::lower_bound(nzs.begin(), nzs.end(), nz[e]) - nzs.begin());
    tab[e].off = L.obs[e];
    tab[e].nz = nz[e];
    tab[e].cls = k;
    b->cls_count[k] += 1;
  }
  b->cls_off.assign(nzs.size() + 1, 0);
  for (size_t k = 0; k < nzs.size(); ++k) b->cls_off[k + 1] = b->cls_off[k] + 4 * nzs[k];
  std::vector<int> ints(3 * (size_t)n_events + 1, 0);
  for (size_t k = 0; k < nzs.size(); ++k) {
    ints[k] = nzs[k];
    ints[n_events + k] = b->cls_off[k];
    ints[2 * n_events + 1 + k] = b->cls_count[k];
  }
  ints[n_events + nzs.size()] = b->cls_off[nzs.size()];
  hipError_t he = hipMemcpyAsync(b->d_avg_ev, tab.data(), tab.size() * sizeof(BatchObsEvent), hipMemcpyHostToDevice,
                                 b->stream);
  if (he == hipSuccess)
    he = hipMemcpyAsync(b->d_cls, ints.data(), ints.size() * sizeof(int), hipMemcpyHostToDevice, b->stream);
  if (he == hipSuccess) he = hipStreamSynchronize(b->stream);
  if (he != hipSuccess) {
    for (auto* x : b->ev) glasma_destroy(x);
    delete b;
    return fail(nullptr, GLASMA_E_HIP, std::string("batch tables: ") + hipGetErrorString(he));
  }
  *out = b;
  return GLASMA_OK;
}

int glasma_batch_classes(const glasma_batch* b, int32_t* n_classes, int32_t* nz_of_class, int32_t* events_of_class) {
  if (!b || !n_classes) return fail(nullptr, GLASMA_E_ARG, "NULL argument");
  *n_classes = (int32_t)b->cls_nz.size();
  for (size_t k = 0; k < b->cls_nz.size(); ++k) {
    if (nz_of_class) nz_of_class[k] = b->cls_nz[k];
    if (events_of_class) events_of_class[k] = b->cls_count[k];
  }
  return GLASMA_OK;
}

int glasma_batch_observe(glasma_batch* b, int32_t n_grid, double* class_avg, double* grid_avg, double* per_event) {
  if (!b) return fail(nullptr, GLASMA_E_ARG, "NULL batch");
  if (!class_avg || !grid_avg) return bfail(b, GLASMA_E_ARG, "class_avg and grid_avg must be device pointers");
  if (n_grid < 1 || n_grid > b->cls_nz.front()) return bfail(b, GLASMA_E_ARG, "need 1 <= n_grid <= the smallest N_z");
  const int n = (int)b->ev.size();
  for (int e = 0; e < n; ++e) {
    glasma_ctx* c = b->ev[e];
    if (!c->ready) return bfail(b, GLASMA_E_STATE, "an event has no state");
    int rc = glasma_observe(c, b->d_obs + b->obs_off[e]);
    if (rc) return bfail(b, rc, std::string("event observables: ") + c->err);
  }
  launch_batch_average(b->d_obs, b->d_avg_ev, n, b->d_cls, b->d_cls + n, b->d_cls + 2 * n + 1,
                       (int)b->cls_nz.size(), b->cls_off.back(), n_grid, class_avg, grid_avg, b->stream);
  BHIPCHK(b, hipGetLastError());
  if (per_event)
    BHIPCHK(b, hipMemcpyAsync(per_event, b->d_obs, (size_t)(b->obs_off.back() + 4 * b->ev.back()->g.nz +
                                                            GLASMA_OBS_NSCALARS) * sizeof(double),
                              hipMemcpyDeviceToDevice, b->stream));
  return GLASMA_OK;
}

int glasma_batch_destroy(glasma_batch* b) {
  if (!b) return GLASMA_OK;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (auto* c : b->ev) glasma_destroy(c);
  delete b;
  return GLASMA_OK;
}

const char* glasma_batch_last_error(const glasma_batch* b) { return b ? b->err.c_str() : g_err.c_str(); }

static int batch_event(glasma_batch* b, int32_t e, glasma_ctx** c) {
  if (!b) return fail(nullptr, GLASMA_E_ARG, "NULL batch");
  if (e < 0 || e >= (int32_t)b->ev.size()) return bfail(b, GLASMA_E_ARG, "event index out of range");
  *c = b->ev[e];
  return GLASMA_OK;
}

int glasma_batch_event(glasma_batch* b, int32_t e, glasma_ctx** ctx) { return batch_event(b, e, ctx); }

// Event table and item map for `bs` sites per item; every event must be at the same step.
static int batch_prepare(glasma_batch* b, int bs, BatchConst* bc) {
  const int64_t s0 = b->ev[0]->step;
  std::vector<EventDesc> tab(b->ev.size());
  std::vector<uint32_t> items;
  for (size_t e = 0; e < b->ev.size(); ++e) {
    glasma_ctx* c = b->ev[e];
    if (!c->ready) return bfail(b, GLASMA_E_STATE, "an event has no state");
    if (c->step != s0) return bfail(b, GLASMA_E_STATE, "events are at different steps");
    EventDesc& d = tab[e];
    d.g = c->g;
    // the buffer current now is current at steps of this parity
    const bool even_now = (s0 & 1) == 0;
    auto rel = [&](void* ptr) { return (uint64_t)((char*)ptr - b->pool); };
    void* cur = c->cur ? c->b.U_alt : c->b.U;
    void* oth = c->cur ? c->b.U : c->b.U_alt;
    d.Ueven = rel(even_now ? cur : oth);
    d.Uodd = rel(even_now ? oth : cur);
    d.E = rel(c->b.E);
    d.rhoA = rel(c->b.rhoA);
    d.rhoB = rel(c->b.rhoB);
    d.item0 = (uint32_t)items.size();
    d.off0 = c->offA;
    d.hops0 = hop_count(c, s0 - 1);
    const uint32_t n = (uint32_t)((c->g.V + bs - 1) / bs);
    for (uint32_t k = 0; k < n; ++k) items.push_back((uint32_t)e);
  }
  BHIPCHK(b, hipMemcpyAsync(b->d_ev, tab.data(), tab.size() * sizeof(EventDesc), hipMemcpyHostToDevice, b->stream));
  BHIPCHK(b, hipMemcpyAsync(b->d_item_event, items.data(), items.size() * sizeof(uint32_t), hipMemcpyHostToDevice,
                            b->stream));
  BHIPCHK(b, hipMemcpyAsync(b->d_ctr, &s0, sizeof(int64_t), hipMemcpyHostToDevice, b->stream));
  BHIPCHK(b, hipStreamSynchronize(b->stream));
  glasma_ctx* c0 = b->ev[0];
  bc->a[0] = b->p.a_T; bc->a[1] = b->p.a_T; bc->a[2] = b->p.a_L;
  bc->dt = b->p.dt;
  bc->hop_p = c0->hop_p;
  bc->hop_q = c0->hop_q;
  bc->reunit_every = b->p.reunit_every;
  bc->items = (uint32_t)items.size();
  return GLASMA_OK;
}

// grid 0: one work-group per item (no loop); grid > 0: that many persistent work-groups
static void batch_launch_one(glasma_batch* b, const BatchConst& bc, int bs, int grid) {
  glasma_ctx* c0 = b->ev[0];
  dispatch(c0, [&]<typename G, typename T>() -> int {
    launch_batch_step<G, T>(b->pool, b->d_ev, b->d_item_event, bc, b->d_ctr, grid, bs, b->stream);
    return 0;
  });
  launch_batch_tick(b->d_ctr, b->stream);
}

// host bookkeeping of every event after n steps
static void batch_advance(glasma_batch* b, int32_t n) {
  for (auto* c : b->ev) {
    const int64_t h = hop_count(c, c->step + n - 1) - hop_count(c, c->step - 1);
    c->offA = (int)((c->offA + h) % c->g.nz);
    c->offB = (int)((c->offB + h) % c->g.nz);
    c->cur = (c->cur + n) & 1;
    c->step += n;
    c->adj_ok = false;
  }
}

int glasma_batch_run(glasma_batch* b, int32_t steps, int32_t graph_chunk) {
  if (!b) return fail(nullptr, GLASMA_E_ARG, "NULL batch");
  if (steps < 0 || graph_chunk < 0) return bfail(b, GLASMA_E_ARG, "steps and graph_chunk must be >= 0");
  if (steps == 0) return GLASMA_OK;
  BatchConst bc;
  int rc = batch_prepare(b, b->bs, &bc);
  if (rc) return rc;
  int32_t done = 0;
  if (graph_chunk > 0 && steps >= graph_chunk) {
    if (!b->exec || b->graph_steps != graph_chunk || b->graph_bs != b->bs || b->graph_grid != b->grid) {
      if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
      if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
      BHIPCHK(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
      for (int32_t k = 0; k < graph_chunk; ++k) batch_launch_one(b, bc, b->bs, b->grid);
      BHIPCHK(b, hipStreamEndCapture(b->stream, &b->graph));
      BHIPCHK(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
      b->graph_steps = graph_chunk;
      b->graph_bs = b->bs;
      b->graph_grid = b->grid;
    }
    // the captured launches carry the item count of this event set and tile size
    while (steps - done >= graph_chunk) {
      BHIPCHK(b, hipGraphLaunch(b->exec, b->stream));
      done += graph_chunk;
    }
  }
  for (; done < steps; ++done) batch_launch_one(b, bc, b->bs, b->grid);
  BHIPCHK(b, hipGetLastError());
  batch_advance(b, steps);
  return GLASMA_OK;
}

int glasma_batch_set_tiling(glasma_batch* b, int32_t sites_per_item, int32_t grid) {
  if (!b) return fail(nullptr, GLASMA_E_ARG, "NULL batch");
  if (sites_per_item != 64 && sites_per_item != 128 && sites_per_item != 256)
    return bfail(b, GLASMA_E_ARG, "sites_per_item must be 64, 128 or 256");
  if (grid < 0) return bfail(b, GLASMA_E_ARG, "grid must be >= 0");
  b->bs = sites_per_item;
  b->grid = grid;
  return GLASMA_OK;
}

// Time every (sites per item, grid) candidate over `steps` steps with HIP events, after one
// untimed step of that candidate (its first launch pays for loading the kernel), and keep
// the fastest; the state advances by steps + candidates * (steps + 1) steps.
int glasma_batch_autotune(glasma_batch* b, int32_t steps, char* report, size_t report_len) {
  if (!b) return fail(nullptr, GLASMA_E_ARG, "NULL batch");
  if (steps < 1) return bfail(b, GLASMA_E_ARG, "steps must be >= 1");
  const int bss[3] = {64, 128, 256};
  const int grids[4] = {0, 4096, 2048, 1024};
  hipEvent_t e0, e1;
  BHIPCHK(b, hipEventCreate(&e0));
  BHIPCHK(b, hipEventCreate(&e1));
  std::string rep = "{\"candidates\": [";
  float best = 1e30f;
  int bb = 256, bg = 0;
  bool first = true;
  // warm-up with the current tiling
  int rc = glasma_batch_run(b, steps, 0);
  if (rc) return rc;
  for (int bs : bss)
    for (int gr : grids) {
      b->bs = bs;
      b->grid = gr;
      rc = glasma_batch_run(b, 1, 0);
      if (rc) return rc;
      BHIPCHK(b, hipEventRecord(e0, b->stream));
      rc = glasma_batch_run(b, steps, 0);
      if (rc) return rc;
      BHIPCHK(b, hipEventRecord(e1, b->stream));
      BHIPCHK(b, hipEventSynchronize(e1));
      float ms = 0.f;
      BHIPCHK(b, hipEventElapsedTime(&ms, e0, e1));
      ms /= (float)steps;
      char buf[128];
      snprintf(buf, sizeof(buf), "%s{\"sites_per_item\": %d, \"grid\": %d, \"ms_per_step\": %.4f}", first ? "" : ", ",
               bs, gr, ms);
      rep += buf;
      first = false;
      if (ms < best) { best = ms; bb = bs; bg = gr; }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->bs = bb;
  b->grid = bg;
  char buf[160];
  snprintf(buf, sizeof(buf), "], \"chosen\": {\"sites_per_item\": %d, \"grid\": %d, \"ms_per_step\": %.4f}}", bb, bg,
           best);
  rep += buf;
  b->tune_report = rep;
  if (report && report_len > 0) {
    std::strncpy(report, rep.c_str(), report_len - 1);
    report[report_len - 1] = 0;
  }
  return GLASMA_OK;
}

// ---- differentiation form ------------------------------------------------------------
// Work buffer of glasma_adjoint_*: [checkpoints: nseg + 1 states][segment: every - 1 states]
// [lam | ebar | rbarA x2 | rbarB x2 | K | loss partials + 1], each part 256-byte aligned.
// A state is [U | E | rho_A | rho_B] in the device layout of the context's precision.
struct AdjRegion {
  size_t sU, sE, sR, state;   // bytes of the state parts and of one state
  int64_t nseg, nslots;       // segments, intermediate states per segment
  size_t ckpt, seg, lam, ebar, rA0, rA1, rB0, rB1, K, part, end;
};
static AdjRegion adj_region(const glasma_params* p, int32_t steps, int32_t every) {
  Geom g = geom_of(p);
  const size_t e = elem(p);
  const int ng = p->nc * p->nc - 1, r = stored_width(p);
  AdjRegion a;
  a.sU = align256(3 * (size_t)r * g.Vp * e);
  a.sE = align256(3 * (size_t)ng * g.Vp * e);
  a.sR = align256((size_t)ng * g.Vp * e);
  a.state = a.sU + a.sE + 2 * a.sR;
  a.nseg = steps > 0 ? (steps + every - 1) / every : 0;
  const int64_t seglen = steps < every ? steps : every;
  a.nslots = seglen > 1 ? seglen - 1 : 0;
  const size_t alg3 = align256(3 * (size_t)ng * g.V * sizeof(double));
  const size_t alg1 = align256((size_t)ng * g.V * sizeof(double));
  a.ckpt = 0;
  a.seg = a.ckpt + (size_t)(a.nseg + 1) * a.state;
  a.lam = a.seg + (size_t)a.nslots * a.state;
  a.ebar = a.lam + alg3;
  a.rA0 = a.ebar + alg3;
  a.rA1 = a.rA0 + alg1;
  a.rB0 = a.rA1 + alg1;
  a.rB1 = a.rB0 + alg1;
  a.K = a.rB1 + alg1;
  a.part = a.K + 2 * alg3;
  a.end = a.part + align256((adj_loss_partials(g) + 1) * sizeof(double));
  return a;
}

struct StatePtr {
  char *U, *E, *rA, *rB;
};
static StatePtr state_at(const AdjRegion& a, char* base) {
  return StatePtr{base, base + a.sU, base + a.sU + a.sE, base + a.sU + a.sE + a.sR};
}

// co-moving charge offset at step s, from the offset off0 at step s0
static int off_at(const glasma_ctx* c, int64_t s0, int off0, int64_t s) {
  const int64_t h = hop_count(c, s - 1) - hop_count(c, s0 - 1);
  return (int)(((off0 + h) % c->g.nz + c->g.nz) % c->g.nz);
}

static int save_state(glasma_ctx* c, const AdjRegion& a, StatePtr d) {
  const size_t e = elem(&c->p);
  HIPCHK(c, hipMemcpyAsync(d.U, c->cur ? c->b.U_alt : c->b.U, 3 * (size_t)c->rs * c->g.Vp * e,
                           hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(d.E, c->b.E, 3 * (size_t)c->ng * c->g.Vp * e, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(d.rA, c->b.rhoA, (size_t)c->ng * c->g.Vp * e, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(d.rB, c->b.rhoB, (size_t)c->ng * c->g.Vp * e, hipMemcpyDeviceToDevice, c->stream));
  (void)a;
  return GLASMA_OK;
}

static int check_adj_args(glasma_ctx* c, int32_t steps, int32_t every) {
  if (!c) return fail(nullptr, GLASMA_E_ARG, "NULL context");
  if (c->p.scheme != 0) return fail(c, GLASMA_E_ARG, "the differentiation form covers the leapfrog scheme");
  if (steps < 0 || every < 1) return fail(c, GLASMA_E_ARG, "steps must be >= 0 and ckpt_every >= 1");
  return GLASMA_OK;
}

int glasma_adjoint_layout(const glasma_params* p, int32_t steps, int32_t ckpt_every, size_t* work_bytes) {
  int rc = check_params(p, nullptr, nullptr);
  if (rc) return rc;
  if (!work_bytes) return fail(nullptr, GLASMA_E_ARG, "work_bytes is NULL");
  if (p->scheme != 0) return fail(nullptr, GLASMA_E_ARG, "the differentiation form covers the leapfrog scheme");
  if (steps < 0 || ckpt_every < 1) return fail(nullptr, GLASMA_E_ARG, "steps must be >= 0 and ckpt_every >= 1");
  *work_bytes = adj_region(p, steps, ckpt_every).end;
  return GLASMA_OK;
}

int glasma_adjoint_forward(glasma_ctx* c, int32_t steps, int32_t ckpt_every, void* work, size_t work_bytes) {
  int rc = check_adj_args(c, steps, ckpt_every);
  if (rc) return rc;
  if (!c->ready) return fail(c, GLASMA_E_STATE, "no state");
  if (!work) return fail(c, GLASMA_E_ARG, "work is NULL");
  const AdjRegion a = adj_region(&c->p, steps, ckpt_every);
  if (work_bytes < a.end) return fail(c, GLASMA_E_ARG, "work buffer smaller than glasma_adjoint_layout");
  char* w = (char*)work;
  const int64_t s0 = c->step;
  const int off0 = c->offA;
  for (int64_t k = 0; k < a.nseg; ++k) {
    if ((rc = save_state(c, a, state_at(a, w + a.ckpt + (size_t)k * a.state)))) return rc;
    const int64_t n = std::min<int64_t>(ckpt_every, steps - k * ckpt_every);
    if ((rc = advance(c, (int32_t)n))) return rc;
  }
  if ((rc = save_state(c, a, state_at(a, w + a.ckpt + (size_t)a.nseg * a.state)))) return rc;
  c->adj_ok = true;
  c->adj_s0 = s0;
  c->adj_steps = steps;
  c->adj_every = ckpt_every;
  c->adj_off0 = off0;
  c->adj_work = work;
  return GLASMA_OK;
}

// The reverse pass of the last glasma_adjoint_forward: seed(...) writes the cotangent of the
// final state into lam, ebar, rbarA, rbarB (plain double arrays in the work buffer), then
// every segment is recomputed from its checkpoint and reversed step by step; the
// cotangents of the starting state are copied out.
template <class Seed>
static int adjoint_reverse(glasma_ctx* c, void* work, size_t work_bytes, Seed&& seed, const double* baseA,
                           const double* baseB, double* dU0, double* dE0, double* drhoA0, double* drhoB0,
                           double* dampA, double* dampB) {
  if (!c->adj_ok || work != c->adj_work || c->step != c->adj_s0 + c->adj_steps)
    return fail(c, GLASMA_E_STATE, "glasma_adjoint_forward with this work buffer must come right before");
  const int32_t steps = c->adj_steps, every = c->adj_every;
  const AdjRegion a = adj_region(&c->p, steps, every);
  if (work_bytes < a.end) return fail(c, GLASMA_E_ARG, "work buffer smaller than glasma_adjoint_layout");
  char* w = (char*)work;
  double* lam = (double*)(w + a.lam);
  double* ebar = (double*)(w + a.ebar);
  double* rA[2] = {(double*)(w + a.rA0), (double*)(w + a.rA1)};
  double* rB[2] = {(double*)(w + a.rB0), (double*)(w + a.rB1)};
  double* K = (double*)(w + a.K);
  double* part = (double*)(w + a.part);
  const double sp[3] = {c->p.a_T, c->p.a_T, c->p.a_L};
  const int64_t s0 = c->adj_s0;
  const int off0 = c->adj_off0;
  auto ckpt = [&](int64_t k) { return state_at(a, w + a.ckpt + (size_t)k * a.state); };
  int cur = 0;
  int rc = dispatch(c, [&]<typename G, typename T>() -> int {
    const StatePtr fin = ckpt(a.nseg);
    int r = seed.template operator()<G, T>(fin, lam, ebar, rA[0], rB[0], part);
    if (r) return r;
    const size_t nE = 3 * (size_t)c->ng * c->g.Vp * sizeof(T), nR = (size_t)c->ng * c->g.Vp * sizeof(T);
    for (int64_t k = a.nseg - 1; k >= 0; --k) {
      const int64_t sk = s0 + k * every;
      const int64_t len = std::min<int64_t>(every, steps - k * every);
      auto slot = [&](int64_t m) {
        if (m == 0) return ckpt(k);
        if (m == len) return ckpt(k + 1);
        return state_at(a, w + a.seg + (size_t)(m - 1) * a.state);
      };
      // recompute the segment's states (bitwise those of the forward pass)
      for (int64_t m = 0; m + 1 < len; ++m) {
        const StatePtr x = slot(m), y = slot(m + 1);
        HIPCHK(c, hipMemcpyAsync(y.E, x.E, nE, hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(y.rA, x.rA, nR, hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(y.rB, x.rB, nR, hipMemcpyDeviceToDevice, c->stream));
        StepConst sc;
        sc.a[0] = sp[0]; sc.a[1] = sp[1]; sc.a[2] = sp[2];
        sc.dt = c->p.dt;
        sc.hop = is_hop(c, sk + m) ? 1 : 0;
        sc.offA = sc.offB = off_at(c, s0, off0, sk + m);
        sc.scheme = 0;
        const bool ru = c->p.reunit_every > 0 && (sk + m + 1) % c->p.reunit_every == 0;
        launch_leapfrog<G, T>((const T*)x.U, (T*)y.U, (T*)y.E, (T*)y.rA, (T*)y.rB, c->g, sc, ru, c->stream);
      }
      for (int64_t m = len - 1; m >= 0; --m) {
        const int64_t s = sk + m;
        const StatePtr x = slot(m), y = slot(m + 1);
        const bool hop = is_hop(c, s);
        launch_adj_step<G, T>((const T*)x.U, (const T*)y.E, (const T*)y.rA, (const T*)x.rB,
                              off_at(c, s0, off0, s + 1), off_at(c, s0, off0, s), hop, c->g, sp, c->p.dt, lam, ebar,
                              K, rA[cur], rB[cur], rA[cur ^ 1], rB[cur ^ 1], c->stream);
        if (hop) cur ^= 1;
      }
    }
    const size_t n3 = 3 * (size_t)c->ng * c->g.V * sizeof(double), n1 = (size_t)c->ng * c->g.V * sizeof(double);
    if (dU0) HIPCHK(c, hipMemcpyAsync(dU0, lam, n3, hipMemcpyDeviceToDevice, c->stream));
    if (dE0) HIPCHK(c, hipMemcpyAsync(dE0, ebar, n3, hipMemcpyDeviceToDevice, c->stream));
    if (drhoA0) HIPCHK(c, hipMemcpyAsync(drhoA0, rA[cur], n1, hipMemcpyDeviceToDevice, c->stream));
    if (drhoB0) HIPCHK(c, hipMemcpyAsync(drhoB0, rB[cur], n1, hipMemcpyDeviceToDevice, c->stream));
    const StatePtr c0 = ckpt(0);
    if (dampA) launch_amp<G, T>(rA[cur], baseA, (const T*)c0.rA, off0, 0, c->g, dampA, c->stream);
    if (dampB) launch_amp<G, T>(rB[cur], baseB, (const T*)c0.rB, off0, 1, c->g, dampB, c->stream);
    return GLASMA_OK;
  });
  if (rc) return rc;
  HIPCHK(c, hipGetLastError());
  return GLASMA_OK;
}

int glasma_adjoint_backward(glasma_ctx* c, int32_t z0, int32_t z1, double scale, void* work, size_t work_bytes,
                            const double* baseA, const double* baseB, double* L, double* dE0, double* drhoA0,
                            double* drhoB0, double* dampA, double* dampB) {
  if (!c) return fail(nullptr, GLASMA_E_ARG, "NULL context");
  if (z0 < 0 || z1 > c->g.nz || z0 >= z1) return fail(c, GLASMA_E_ARG, "need 0 <= z0 < z1 <= nz");
  const double sp[3] = {c->p.a_T, c->p.a_T, c->p.a_L};
  double* Lout = nullptr;
  // the slab energy's own cotangent as the seed
  auto seed = [&]<typename G, typename T>(const StatePtr& fin, double* lam, double* ebar, double* rA, double* rB,
                                          double* part) -> int {
    Lout = part + adj_loss_partials(c->g);
    launch_adj_loss<G, T>((const T*)fin.U, (const T*)fin.E, c->g, sp, z0, z1, scale, lam, ebar, rA, rB, part, Lout,
                          c->stream);
    return GLASMA_OK;
  };
  int rc = adjoint_reverse(c, work, work_bytes, seed, baseA, baseB, nullptr, dE0, drhoA0, drhoB0, dampA, dampB);
  if (rc) return rc;
  if (L) {
    HIPCHK(c, hipMemcpyAsync(L, Lout, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return GLASMA_OK;
}

int glasma_adjoint_backward_cotangent(glasma_ctx* c, void* work, size_t work_bytes, const double* lamU,
                                      const double* ebarE, const double* rbarA, const double* rbarB,
                                      const double* baseA, const double* baseB, double* dU0, double* dE0,
                                      double* drhoA0, double* drhoB0, double* dampA, double* dampB) {
  if (!c) return fail(nullptr, GLASMA_E_ARG, "NULL context");
  const size_t n3 = 3 * (size_t)c->ng * c->g.V, n1 = (size_t)c->ng * c->g.V;
  auto seed = [&]<typename G, typename T>(const StatePtr&, double* lam, double* ebar, double* rA, double* rB,
                                          double*) -> int {
    auto put = [&](double* dst, const double* src, size_t n) -> int {
      if (src) HIPCHK(c, hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
      else launch_zero(dst, (int)n, c->stream);
      return GLASMA_OK;
    };
    int r;
    if ((r = put(lam, lamU, n3)) || (r = put(ebar, ebarE, n3)) || (r = put(rA, rbarA, n1)) || (r = put(rB, rbarB, n1)))
      return r;
    return GLASMA_OK;
  };
  return adjoint_reverse(c, work, work_bytes, seed, baseA, baseB, dU0, dE0, drhoA0, drhoB0, dampA, dampB);
}

int glasma_slab_energy(glasma_ctx* c, int32_t z0, int32_t z1, double* L) {
  if (!c || !L) return fail(c, GLASMA_E_ARG, "NULL argument");
  if (!c->ready) return fail(c, GLASMA_E_STATE, "no state");
  if (z0 < 0 || z1 > c->g.nz || z0 >= z1) return fail(c, GLASMA_E_ARG, "need 0 <= z0 < z1 <= nz");
  const double sp[3] = {c->p.a_T, c->p.a_T, c->p.a_L};
  double* part = (double*)c->b.work;
  double* out = part + adj_loss_partials(c->g);
  dispatch(c, [&]<typename G, typename T>() -> int {
    launch_adj_loss<G, T>(cur_U<T>(c), (const T*)c->b.E, c->g, sp, z0, z1, 1.0, nullptr, nullptr, nullptr, nullptr,
                          part, out, c->stream);
    return 0;
  });
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipMemcpyAsync(L, out, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return GLASMA_OK;
}

int glasma_set_state_device(glasma_ctx* c, const double* U, const double* E, const double* rhoA, const double* rhoB,
                            const double* ampA, const double* ampB, int64_t step0) {
  if (!c || !U || !E || !rhoA || !rhoB) return fail(c, GLASMA_E_ARG, "NULL argument");
  if (step0 < 0) return fail(c, GLASMA_E_ARG, "step0 must be >= 0");
  dispatch(c, [&]<typename G, typename T>() -> int {
    launch_pack_links<G, T>(U, (T*)c->b.U, c->g, c->stream);
    launch_pack<G, T>(E, nullptr, (T*)c->b.E, c->g, 3, c->ng, c->stream);
    launch_pack<G, T>(rhoA, ampA, (T*)c->b.rhoA, c->g, 1, c->ng, c->stream);
    launch_pack<G, T>(rhoB, ampB, (T*)c->b.rhoB, c->g, 1, c->ng, c->stream);
    return 0;
  });
  HIPCHK(c, hipGetLastError());
  c->cur = 0;
  c->offA = c->offB = 0;
  c->step = step0;
  c->ready = true;
  c->semi_prev = false;
  c->adj_ok = false;
  return GLASMA_OK;
}

int glasma_get_state_device(glasma_ctx* c, double* U, double* E, double* rhoA, double* rhoB) {
  if (!c) return fail(nullptr, GLASMA_E_ARG, "NULL context");
  if (!c->ready) return fail(c, GLASMA_E_STATE, "no state");
  dispatch(c, [&]<typename G, typename T>() -> int {
    if (U) launch_unpack_links<G, T>(cur_U<T>(c), U, c->g, c->stream);
    if (E) launch_unpack<G, T>((const T*)c->b.E, E, c->g, 3, c->ng, 0, 0, c->stream);
    if (rhoA) launch_unpack<G, T>((const T*)c->b.rhoA, rhoA, c->g, 1, c->ng, c->offA, 1, c->stream);
    if (rhoB) launch_unpack<G, T>((const T*)c->b.rhoB, rhoB, c->g, 1, c->ng, c->offB, 2, c->stream);
    return 0;
  });
  HIPCHK(c, hipGetLastError());
  return GLASMA_OK;
}
