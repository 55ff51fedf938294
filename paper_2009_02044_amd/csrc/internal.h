// Internal declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "lattice.h"

namespace gl {

// reunit: the step also reunitarises the new links (as launch_reunit would after it)
template <typename G, typename T>
void launch_leapfrog(const T* U, T* Unew, T* E, T* rhoA, T* rhoB, const Geom& g, const StepConst& c,
                     bool reunit, hipStream_t st);

// Batched form (step.hip): one descriptor per event, work items of blockDim.x sites.
// Buffers are byte offsets into the batch's pool, whose base is a kernel argument (so
// the compiler knows every access is to device memory).
struct EventDesc {
  Geom g;
  uint64_t Ueven;     // link buffer that is current at even steps
  uint64_t Uodd;      // link buffer that is current at odd steps
  uint64_t E;
  uint64_t rhoA;
  uint64_t rhoB;
  uint32_t item0;     // first work item of the event
  int32_t off0;       // charge offset at the reference step
  int64_t hops0;      // hop count S(s_ref - 1) at the reference step
};
struct BatchConst {
  double a[3];
  double dt;
  int64_t hop_p, hop_q;  // dt / a_L = hop_p / hop_q
  int reunit_every;
  uint32_t items;
};
template <typename G, typename T>
void launch_batch_step(char* pool, const EventDesc* ev, const uint32_t* item_event, const BatchConst& bc,
                       const int64_t* ctr, int grid, int bs, hipStream_t st);
void launch_batch_tick(int64_t* ctr, hipStream_t st);

// Observables at the current integer time, written to `out` (device, double):
// [0, 4 nz): transverse means eps, p_L, p_T, S_L per layer; then OBS_* scalars.  En: E(t + dt/2)
// from the semi-implicit solve of the next step (null: the leapfrog update, computed here).
enum {
  OBS_ENERGY = 0, OBS_GAUSS_L2, OBS_RHO_L2, OBS_GAUSS_MAX, OBS_UNITARITY, OBS_NONFINITE,
  OBS_GAUSS_REL, OBS_NSCALARS = 8
};
template <typename G, typename T>
void launch_observe(const T* U, const T* E, const T* rhoA, const T* rhoB, const T* En, const Geom& g,
                    const StepConst& c, double* partial, double* out, hipStream_t st);
size_t observe_partial_doubles(const Geom& g);
// address (for `device`) and size in doubles of the file-scope partial-sum array used by the
// allocation-free observables call
hipError_t observe_static_scratch(int device, double** ptr, size_t* capacity);
// Observing step (FP64 leapfrog, nt a multiple of 64): the Gauss residual kernel runs on
// the state before the step, the step kernel adds the energy slots, then the finish pass.
bool fused_observe_geometry(const Geom& g);
int fused_observe_blocks_per_layer(const Geom& g);
template <typename G, typename T>
void launch_obs_gauss(const T* U, const T* E, const T* rhoA, const T* rhoB, const Geom& g, const StepConst& c,
                      double* partial, hipStream_t st);
template <typename G, typename T>
void launch_leapfrog_observe(const T* U, T* Unew, T* E, T* rhoA, T* rhoB, const Geom& g, const StepConst& c,
                             double* partial, hipStream_t st);
void launch_observe_finish(const double* partial, int nbx, const Geom& g, const StepConst& c, double* out,
                           hipStream_t st);
// Observing step around a plain leapfrog step (any geometry and precision): launch_obs_pre on
// the state before the step (partial sums as launch_observe; Q: obs_split_scratch_elems
// reals of the state's precision), the step, then launch_obs_post (partial sums completed
// and finished into out).
size_t obs_split_scratch_elems(const Geom& g, int ng);
template <typename G, typename T>
void launch_obs_pre(const T* U, const T* E, const T* rhoA, const T* rhoB, const Geom& g, const StepConst& c, T* Q,
                    double* partial, hipStream_t st);
template <typename G, typename T>
void launch_obs_post(const T* E, const T* Q, const Geom& g, const StepConst& c, double* partial, double* out,
                     hipStream_t st);
// event averages of a batch's observables (class averages per N_z, common z / N_z grid)
struct BatchObsEvent {
  int64_t off;   // doubles from the start of the observables region
  int nz;
  int cls;       // index of the event's N_z class
};
void launch_batch_average(const double* obs, const BatchObsEvent* ev, int n_events, const int* cls_nz,
                          const int* cls_off, const int* cls_count, int n_cls, int cls_total, int n_grid,
                          double* cls_out, double* grid_out, hipStream_t st);
// local rest frame per layer from the observe slices (2 * nz doubles out)
void launch_rest_frame(const double* obs, int nz, double* out, hipStream_t st);

template <typename G, typename T>
void launch_current(const T* U, const T* rhoA, const T* rhoB, const Geom& g, const StepConst& c,
                    T* j, hipStream_t st);

template <typename G, typename T>
void launch_reunit(T* U, const Geom& g, hipStream_t st);

// Semi-implicit scheme (semi.hip)
// f1(Uc, Uo) of every link into out; cache (may be null): the marching pass also stores
// the loops of Uc alone there for the iterations of the step
template <typename G, typename T>
void launch_semi_f1(const T* Uc, const T* Uo, T* out, const Geom& g, const StepConst& c, hipStream_t st,
                    T* cache = nullptr);
template <typename G, typename T>
void launch_semi_begin(const T* U, const T* E, const T* Ep, const T* J, T* Up, T* Ut, T* Et, const Geom& g,
                       const StepConst& c, hipStream_t st);
template <typename G, typename T>
void launch_semi_keep(const T* E, const T* J, T* Ep, const Geom& g, hipStream_t st);
// hop of the charges with U(t): commit = false writes only the current a_L (rho_A' - rho_B) into J,
// commit = true moves the charges (after the solve has converged)
template <typename G, typename T>
void launch_semi_hop(const T* U, T* rhoA, T* rhoB, T* J, bool commit, const Geom& g, const StepConst& c,
                     hipStream_t st);
// Ebase = E + dt F2 + [z] J in place over F2 (J: dt j_z on hop steps, or null)
template <typename G, typename T>
void launch_semi_base(const T* E, T* F2, const T* J, const Geom& g, double dt, hipStream_t st);
// one fixed-point iteration E' = Ebase + dt f1(Uc, Ut_in); conv (2 doubles, zeroed before)
// receives max|dE|, max|E|; with conv_prev (the slot of the iteration before) already
// converged to tol it does nothing
template <typename G, typename T>
void launch_semi_iter(const T* Uc, const T* Ut_in, const T* Ebase, T* Et, T* Ut_out, double* conv,
                      const double* conv_prev, double tol, const Geom& g, const StepConst& c, hipStream_t st,
                      const T* cache);
// The marching pass (semi_march.hip) for lattices with 8 <= nt <= 64, nt dividing 64:
// mode 0 writes f1(A, B) to it.F; mode 1 is one fixed-point iteration (A = U(t), B = the
// trial links) with the fields of it.
struct MarchIter {
  const void* Ebase;
  void* Et;
  void* Ut_out;
  double* conv;
  const double* conv_prev;
  double tol, omega;
  void* F;
  void* cache;   // loops of slice A alone: written by mode 0 (if not null), read by mode 1
};
// elements of the loop cache: 3 planes of full matrices (18 or 4 reals) per padded site
size_t march_cache_elems(const Geom& g, int nc);
bool march_geometry(const Geom& g);
template <typename G, typename T>
void launch_semi_march(const T* A, const T* B, const Geom& g, const StepConst& c, int mode, const MarchIter& it,
                       hipStream_t st);
void launch_zero(double* p, int n, hipStream_t st);
template <typename G, typename T>
void launch_copy(const T* src, T* dst, int64_t n, hipStream_t st);

// Initial conditions.  launch_ic_phi: the transverse charges of one sheet of both
// nuclei (double, [2][NG][nt*nt]: A then B, at the start of work; work needs
// ic_work_doubles(g, NG) doubles) -> their fields phi, written to phi_out in the same
// layout.  launch_ic_fields: links, E and charges from the fields of ns sheets
// (phi: [ns][2][NG][nt*nt], sheet 0 the leading edge of each nucleus).
struct McvConst {
  double m_ir, uv_cut, sigma, zA, zB;
};
size_t ic_work_doubles(const Geom& g, int ng);
void launch_ic_phi(double* work, double* phi_out, int ng, const Geom& g, const StepConst& c, const McvConst& mv,
                   hipStream_t st);
template <typename G, typename T>
void launch_ic_fields(const double* phi, int ns, T* U, T* E, T* rhoA, T* rhoB, const Geom& g, const StepConst& c,
                      const McvConst& mv, hipStream_t st);
// Boost-invariant tau = 0+ fields: work = [initial-condition DFT region | V of both
// nuclei (2 nt^2 links of double) | block sums]; bi_work_doubles gives its size.
size_t bi_work_doubles(const Geom& g, int ng, size_t link_doubles);
template <int NC>
void launch_bi_sheet(const double* phi, double* work_links, const Geom& g, int first, hipStream_t st);
template <int NC>
void launch_bi_fields(const double* work_links, double* partial, const Geom& g, double a_T, double* Ez, double* Bz,
                      double* out3, hipStream_t st);
// charges from the (modified) Gauss law: rho = D.(E + scale F2), F2 may be null; split at nz/2
template <typename G, typename T>
void launch_gauss_charges(const T* U, const T* E, const T* F2, double scale, T* rhoA, T* rhoB, const Geom& g,
                          const StepConst& c, hipStream_t st);

// Differentiation form (adjoint.hip): cotangents in double, plain [dir][a][V] arrays.
// Loss of layers [z0, z1) of the state (U, E) into out[0] (partial needs adj_loss_partials
// doubles); with lam != null also the seed cotangents scale * dL/d(state).
size_t adj_loss_partials(const Geom& g);
template <typename G, typename S>
void launch_adj_loss(const S* U, const S* E, const Geom& g, const double* a, int z0, int z1, double scale,
                     double* lam, double* ebar, double* rA, double* rB, double* partial, double* out, hipStream_t st);
// One reverse step: state s (U0, rhoB0 at offset offB0), E1 and rhoA1 (offset offA1) of
// state s + 1; K holds 6 n_g V doubles; on hop steps the charge cotangents move from
// (rAin, rBin) to (rAout, rBout).
template <typename G, typename S>
void launch_adj_step(const S* U0, const S* E1, const S* rhoA1, const S* rhoB0, int offA1, int offB0, bool hop,
                     const Geom& g, const double* a, double dt, double* lam, double* ebar, double* K,
                     const double* rAin, const double* rBin, double* rAout, double* rBout, hipStream_t st);
template <typename G, typename S>
void launch_pack(const double* src, const double* amp, S* dst, const Geom& g, int ndir, int width, hipStream_t st);
template <typename G, typename S>
void launch_unpack(const S* src, double* dst, const Geom& g, int ndir, int width, int off, int kind, hipStream_t st);
template <typename G, typename S>
void launch_pack_links(const double* src, S* dst, const Geom& g, hipStream_t st);
template <typename G, typename S>
void launch_unpack_links(const S* src, double* dst, const Geom& g, hipStream_t st);
template <typename G, typename S>
void launch_amp(const double* rbar, const double* base, const S* rho, int off, int which, const Geom& g, double* out,
                hipStream_t st);

}  // namespace gl
