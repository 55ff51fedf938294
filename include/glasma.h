/*
 * glasma.h -- C-ABI of the MI355X (gfx950) library for the 3+1D Glasma
 * colored-particle-in-cell (CPIC) evolution of Ipp & Mueller, "Progress on 3+1D
 * Glasma simulations" (arXiv:2009.02044).
 *
 * The library evolves SU(2) or SU(3) gauge links U_i(x) and Lie-algebra electric
 * fields E_i(x) on an nz x nt x nt lattice (z = beam axis, periodic in all three
 * directions), driven by the colour charges of two nuclei that move at the speed of
 * light along -z (nucleus A) and +z (nucleus B).
 *
 * Conventions (lattice units; the coupling g is absorbed into the fields):
 *   spacings a_x = a_y = a_T, a_z = a_L; time step dt with dt/a_L rational in (0, 1].
 *   site index s = (z * nt + y) * nt + x; V = nz * nt * nt.
 *   Generators t^a = sigma^a/2 (SU(2)) or lambda^a/2 (SU(3)); n_g = nc^2 - 1.
 *   Algebra fields are stored by components X^a = 2 Tr(t^a X).
 *   E_i and j_i are the continuum-normalised fields: the paper's E and j in
 *   eqs. lattice_1/2 (Sec. 3) equal a_i E_i and a_i j_i.  One step is
 *     E_i(t+dt/2) = E_i(t-dt/2) + dt [ -(1/a_i) sum_{j!=i} a_j^-2 P(U_{i,j} + U_{i,-j}) + j_i ]
 *     U_i(t+dt)   = exp(i a_i dt E_i(t+dt/2)) U_i(t)
 *   with P(M) the hermitian traceless part of (M - M^dag)/(2i) (the paper's [M]_ah is
 *   i P(M)), and the Gauss law (eq. gauss) reads
 *     sum_i [E_i(x) - U_i^dag(x-i) E_i(x-i) U_i(x-i)] / a_i = rho_A(x) + rho_B(x).
 *
 * Host array layout (all host arrays are double, structure of arrays):
 *   links  U[i][c][s], i = 0:x 1:y 2:z; SU(2): c = 0..3, U = u0 + i (u1 s1 + u2 s2 + u3 s3);
 *          SU(3): c = 2 (3 r + k) + {0 Re, 1 Im} for matrix entry (r, k)
 *   E      E[i][a][s];  charges rho[a][s] at their physical lattice positions.
 * Device buffers hold the same fields in the context's precision (fp = 64: double,
 * fp = 32: float) in a tiled layout: per direction, records of 64 consecutive sites
 * in which the components are grouped in 16-byte chunks, one row of 64 chunks per
 * group; the site count is padded to Vp = 64 ceil(V/64).  SU(3) links are stored by
 * their first two rows (r_S = 12 reals; the third row of a special unitary matrix is
 * conj(row 0 x row 1) and is rebuilt on every load), SU(2) links by r_S = 4 reals.  The
 * charge buffers are stored co-moving with their nucleus.  Read and write device state
 * only through glasma_init_state / glasma_get_state (or their device-array variants).
 *
 * Memory: the caller allocates every device buffer (sizes from glasma_layout) and
 * keeps it alive until glasma_destroy; the library never allocates or frees device
 * memory itself.  The context holds only host metadata.
 * Streams: all device work is enqueued on the stream given to glasma_create; calls
 * return without waiting unless stated otherwise.
 * Errors: every call returns GLASMA_OK (0) or a negative code; no exception crosses
 * the ABI.  glasma_last_error(ctx) (or NULL for failures without a context) gives
 * a message.  A context is not thread safe.
 */
#ifndef GLASMA_H
#define GLASMA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GLASMA_OK 0
#define GLASMA_E_ARG (-1)        /* invalid argument or size */
#define GLASMA_E_HIP (-2)        /* HIP runtime error (message kept) */
#define GLASMA_E_NONFINITE (-3)  /* NaN / Inf found in the fields */
#define GLASMA_E_CONSTRAINT (-4) /* Gauss residual above the requested bound */
#define GLASMA_E_NOCONV (-5)     /* semi-implicit iteration reached max_iter */
#define GLASMA_E_STATE (-6)      /* call out of order (e.g. step before init) */

typedef struct glasma_ctx glasma_ctx;

typedef struct {
  int32_t nc;           /* 2 or 3: gauge group SU(nc) */
  int32_t nz, nt;       /* lattice nz (beam axis) x nt x nt; nz >= 2, nt >= 2 */
  double a_T, a_L, dt;  /* spacings and time step, dt/a_L rational in (0, 1] */
  int32_t fp;           /* 64 or 32: storage and arithmetic precision of U, E, rho */
  int32_t scheme;       /* 0: leapfrog (eqs. lattice_1/2); 1: semi-implicit (Sec. 3) */
  int32_t reunit_every; /* > 0: reunitarise links (FP64 arithmetic) every k steps */
  int32_t max_iter;     /* semi-implicit: fixed-point iteration cap */
  double tol;           /* semi-implicit: convergence bound on max |dE| / max |E| */
} glasma_params;

/* Device buffers (caller-owned; sizes in bytes from glasma_layout, same order). */
typedef struct {
  void* U;      /* links at the current time, 3 * r_S * Vp reals (r_S = 4 or 12) */
  void* U_alt;  /* second link buffer of the same size (the step writes into it) */
  void* E;      /* electric field, 3 * n_g * Vp reals */
  void* rhoA;   /* charges of nucleus A, n_g * Vp reals (co-moving storage) */
  void* rhoB;   /* charges of nucleus B, n_g * Vp reals (co-moving storage) */
  void* work;   /* scratch: initial conditions, reductions, parked plaquette projections, iterations */
} glasma_buffers;

/* Initial-condition parameters (Sec. 2 Poisson solution; Sec. 3 eq. single_sheet). */
typedef struct {
  double m_ir;    /* IR regulator m of the transverse Poisson equation (> 0) */
  double uv_cut;  /* UV cutoff Lambda on |k~| (<= 0: none) */
  double sigma;   /* width of the Gaussian longitudinal profile (units of length) */
  double zA, zB;  /* centres of nucleus A (moving -z) and B (moving +z) at t0 */
} glasma_mv;

/* Number of doubles glasma_observe writes: 4 * nz slices + GLASMA_OBS_NSCALARS. */
#define GLASMA_OBS_NSCALARS 8
/* Scalar slots after the 4 * nz slices (eps, p_L, p_T, S_L per layer, each the
 * transverse mean at that layer). */
#define GLASMA_OBS_ENERGY 0      /* H = a_T^2 a_L sum_x eps */
#define GLASMA_OBS_GAUSS_L2 1    /* ||G||_2 over all sites and colours */
#define GLASMA_OBS_RHO_L2 2      /* ||rho||_2 */
#define GLASMA_OBS_GAUSS_MAX 3   /* max_x,a |G^a(x)| */
#define GLASMA_OBS_UNITARITY 4   /* max over links of |U^dag U - 1| and |det U - 1| */
#define GLASMA_OBS_NONFINITE 5   /* number of sites with a NaN / Inf */
#define GLASMA_OBS_GAUSS_REL 6   /* ||G||_2 / ||rho||_2 (||G||_2 if rho = 0) */

/* Library version string. */
const char* glasma_version(void);

/* Message of the last failure on ctx (NULL: the last failure without a context). */
const char* glasma_last_error(const glasma_ctx* ctx);

/* Byte sizes of the six glasma_buffers entries for params p (bytes[6]). */
int glasma_layout(const glasma_params* p, size_t* bytes);

/* Create a context over caller-owned device buffers b on HIP stream `stream`
 * (a hipStream_t; NULL = default stream).  The buffers are not read here. */
int glasma_create(const glasma_params* p, const glasma_buffers* b, void* stream, glasma_ctx** out);

/* Destroy the context (host memory only; the caller frees its buffers). */
int glasma_destroy(glasma_ctx* ctx);

/* Upload a state from host double arrays in the layout above (charges at physical
 * positions).  The state is U(t), E(t - dt/2), rho(t - dt/2) with t = t0 + step0 dt;
 * step0 fixes the phase of the charge hop schedule.  Synchronous. */
int glasma_init_state(glasma_ctx* ctx, const double* U, const double* E, const double* rhoA,
                      const double* rhoB, int64_t step0);

/* Build the MV initial state on the GPU (Sec. 2 and 3) from the transverse colour
 * charges rhoT_A, rhoT_B (host double, [n_g][nt][nt] each; the random draw of the
 * MV ensemble is an input).  Sets step = 0.  Asynchronous after the upload. */
int glasma_init_mv(glasma_ctx* ctx, const glasma_mv* mv, const double* rhoT_A, const double* rhoT_B);

/* Nuclei whose colour structure varies along the beam axis (Sec. 3 allows charge
 * densities rho(x^+-, x_T) beyond eq. single_sheet; Sec. 5 names the stack of
 * uncorrelated sheets): each nucleus is cut into ns pieces of equal weight of its
 * Gaussian profile, piece k carrying the transverse charges of sheet k, and the
 * Wilson line of Sec. 2 is the path-ordered product
 *   V = exp(-i lambda_0 phi_0) ... exp(-i lambda_{ns-1} phi_{ns-1}),
 *   lambda_k = clamp(ns Lambda - k, 0, 1)   (Lambda: the profile's cumulative weight),
 * sheet 0 the leading edge (largest z for B, smallest for A), each later sheet to the
 * right (so that, with A_i = V d_i V^dag / (ig), the field inside piece k is sheet k's
 * own rotated by the completed pieces).  rhoT_A, rhoT_B: host
 * double, [ns][n_g][nt][nt] (for the MV ensemble of one sheet with variance mu^2, draw
 * each sheet with mu^2 / ns).  ns = 1 is glasma_init_mv.  For ns > 1 the sheets' fields
 * are staged in the second link buffer: ns * 2 * n_g * nt^2 doubles must fit there
 * (ns <= nz always does), else GLASMA_E_ARG.  Sets step = 0.  Asynchronous after the
 * uploads (the host arrays may be released on return). */
int glasma_init_mv_sheets(glasma_ctx* ctx, const glasma_mv* mv, int32_t ns, const double* rhoT_A,
                          const double* rhoT_B);

/* Boost-invariant Glasma at tau = 0+ (Sec. 2, eqs. glasma_ic1, glasma_ic2, LC_gauge1): the
 * longitudinal fields that infinitely thin nuclei with these transverse charges leave at
 * the boundary of the forward light cone, the reference that thin nuclei approach at
 * mid-rapidity.  With alpha^i_N = P(V_N(x) V_N^dag(x + i)) / a_T on the transverse links
 * (V_N the Wilson line behind nucleus N: exp(-i phi_N), or the ordered product over ns
 * sheets as in glasma_init_mv_sheets; P the hermitian traceless part of
 * (W - W^dag)/(2i)) and g = 1:
 *   E_z = -i [alpha_A^i, alpha_B^i]  (at the sites, each commutator averaged over the two
 *          links of direction i that meet there),
 *   B_z = -i ([alpha_A^x, alpha_B^y] - [alpha_A^y, alpha_B^x])  (at the xy plaquette
 *          centres, alpha^x averaged over the plaquette's x links, alpha^y over its y links).
 * p: nc, nt and a_T are used (the other fields must be valid); mv: m_ir, uv_cut (sigma,
 * zA, zB unused).  rhoT_A, rhoT_B: host double, [ns][n_g][nt][nt].  work: device scratch
 * of glasma_bi_work_bytes bytes.  Ez, Bz: device double [n_g][nt][nt] (component-major,
 * Bz(x) belongs to the plaquette at x, x + e_x, x + e_x + e_y, x + e_y); out3: device
 * double[3] = transverse means (eps_0, E_z^2/2, B_z^2/2), |X|^2 = sum_a X^a X^a.
 * Asynchronous on `stream` (a hipStream_t; NULL = default) after the uploads. */
int glasma_bi_work_bytes(const glasma_params* p, size_t* bytes);
int glasma_bi_fields(const glasma_params* p, const glasma_mv* mv, int32_t ns, const double* rhoT_A,
                     const double* rhoT_B, void* work, double* Ez, double* Bz, double* out3, void* stream);

/* Advance n >= 0 steps (leapfrog or semi-implicit per params, CPIC hops on the steps
 * the schedule S(s) = floor((s + 1/2) dt/a_L + 1/2) advances, reunitarisation every
 * reunit_every steps when set).  Asynchronous for the leapfrog.  The semi-implicit step
 * iterates its fixed point (under-relaxed) until max|dE| <= tol max|E|, from a start
 * extrapolated from the previous step when the context made that step; after a state
 * upload it starts from E, so a resumed run agrees with an uninterrupted one to tol.  Its
 * iterations are enqueued in batches that test convergence on the device; the host waits
 * once per batch (usually once per step).  GLASMA_E_NOCONV after max_iter iterations,
 * GLASMA_E_NONFINITE on a non-finite field; either leaves the state (links, E, charges,
 * step counter) as it was before the failed step, so the context stays consistent. */
int glasma_step(glasma_ctx* ctx, int32_t n);

/* Current j (device, 3 * n_g * V reals of the context's precision, in the plain host
 * layout j[i][a][s] -- not the tiled device layout of E) that
 * the next step deposits: j_z = (a_L/dt)(rho_A' - rho_B) on hop steps (rho_A' is
 * the transported A charge), zero otherwise (Sec. 3, eq. continuity).  Does not
 * change the state.  Asynchronous. */
int glasma_deposit_current(glasma_ctx* ctx, void* j_out);

/* Observables at the current integer time into device memory d_out (double,
 * 4 * nz + GLASMA_OBS_NSCALARS): eps, p_L, p_T, S_L slices (Sec. 4, <T^{mu nu}> and
 * eq. pT_eL) computed in double precision, then the scalars listed above.  Electric terms
 * average the two half steps, E^2 = (|E(t - dt/2)|^2 + |E(t + dt/2)|^2)/2 and
 * Ebar = (E(t - dt/2) + E(t + dt/2))/2 in S_L, for both schemes: the leapfrog's E(t + dt/2)
 * is computed here; the semi-implicit scheme's comes from solving the next step (that solve
 * is discarded; the call then waits for it and fails like glasma_step).  Magnetic terms
 * are the plain plaquettes at t for both schemes, so for the semi-implicit scheme H is the
 * Wilson-action energy, not the conserved energy of its modified action.  The Gauss slots
 * hold the standard residual at (U(t), E(t - dt/2), rho(t - dt/2)).  Does not change the
 * state.  Asynchronous for the leapfrog. */
int glasma_observe(glasma_ctx* ctx, double* d_out);

/* glasma_observe for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same observables,
 * bitwise, with the per-block partial sums held in a file-scope device array of the library
 * (4 MiB per GPU the library runs on, kept until the process ends) instead of the context's
 * work buffer.  The call allocates and frees nothing (no hipMalloc, no library routine that
 * allocates); the first call on a device looks the array's address up for it.  Every call
 * on one GPU shares that array and each call writes every partial it reads, so nothing
 * needs clearing; calls that overlap on one GPU (several streams or host threads) race.
 * Limits: the leapfrog scheme (scheme 1: GLASMA_E_ARG), and lattices whose partial sums
 * (nz ceil(nt^2 / 256) work-groups x 9 doubles) fit in the array, up to 524288 doubles
 * (512 x 64 x 64 needs 73728; larger: GLASMA_E_ARG with the sizes).  Asynchronous. */
int glasma_observe_noalloc(glasma_ctx* ctx, double* d_out);

/* n >= 1 steps, writing to d_out (device, as glasma_observe) the observables of the state
 * the last step starts from: the same as glasma_step(n - 1), glasma_observe,
 * glasma_step(1), up to rounding, without forming the force twice.  Leapfrog: a pass over
 * the state before the last step sums what that state fixes (Gauss residual, B^2, the
 * E(t - dt/2) halves of E^2 and S_L, unitarity) and parks two plaquette projections in the
 * work buffer; after the step a second pass adds the E(t + dt/2) halves, E(t + dt/2) being
 * the step's own (for FP32 storage its FP32 update).  For FP64 with nt a multiple of 64 the
 * step kernel itself adds the energy slots after a Gauss-residual pass.  An event of a batch
 * has no room for the parked projections and runs glasma_observe, then the step.  The non-finite
 * slot counts detections (a site may count twice).  For the semi-implicit scheme the
 * observables pass runs between the last step's converged solve and its commit (one solve,
 * not two).  Asynchronous for the leapfrog; errors as glasma_step. */
int glasma_step_observe(glasma_ctx* ctx, int32_t n, double* d_out);

/* Local rest frame of every layer (Sec. 4: the local energy density from diagonalising
 * the energy-momentum tensor).  Reads the slices that glasma_observe wrote to d_obs
 * (device, 4 * nz + GLASMA_OBS_NSCALARS doubles) and writes to d_out (device, 2 * nz
 * doubles, caller-owned): eps_loc[z], the eigenvalue of the timelike eigenvector of the
 * (t, z) block [[eps, -S_L], [S_L, -p_L]] of T^mu_nu, then v[z], that eigenvector's
 * velocity along +z:
 *   eps_loc = ((eps - p_L) + sqrt((eps + p_L)^2 - 4 S_L^2)) / 2,
 *   v = 2 S_L / ((eps + p_L) + sqrt((eps + p_L)^2 - 4 S_L^2))
 * (the square root of a negative round-off is taken as 0; v = 0 where eps + p_L = 0).
 * Asynchronous on the context's stream; GLASMA_E_ARG for NULL pointers. */
int glasma_rest_frame(glasma_ctx* ctx, const double* d_obs, double* d_out);

/* Synchronous variant to host memory: tmunu_z [4][nz] (may be NULL) and scalars
 * (each may be NULL). */
int glasma_observables(glasma_ctx* ctx, double* tmunu_z, double* gauss_rel, double* gauss_max,
                       double* energy, double* unitarity_max);

/* Download the state to host double arrays (layout above; charges at physical
 * positions; any pointer may be NULL) and the step counter.  Synchronous. */
int glasma_get_state(glasma_ctx* ctx, double* U, double* E, double* rhoA, double* rhoB,
                     int64_t* step);

/* Project every link back onto SU(nc) in double arithmetic (SU(2): q/|q|; SU(3):
 * Gram-Schmidt of rows 1, 2, row 3 = conj(r1 x r2)).  Asynchronous. */
int glasma_reunitarize(glasma_ctx* ctx);

/* Fixed-point iterations used by the last semi-implicit step (host value). */
int glasma_last_iterations(const glasma_ctx* ctx, int32_t* iters);

/* Current step counter (host value). */
int glasma_get_step(const glasma_ctx* ctx, int64_t* step);

/* ---- Device state transfer ---------------------------------------------------
 * Same layout as glasma_init_state / glasma_get_state, but the arrays are device
 * memory (double): U [3][r_U][V], E [3][n_g][V], rho [n_g][V] at physical positions. */

/* Set the state from device arrays; ampA / ampB (device, [V], may be NULL = 1) scale the
 * charges of each cell: rho(x) -> amp(x) rho(x).  Resets the step counter to step0 and the
 * charge storage to offset 0.  Asynchronous. */
int glasma_set_state_device(glasma_ctx* ctx, const double* U, const double* E, const double* rhoA,
                            const double* rhoB, const double* ampA, const double* ampB, int64_t step0);

/* Write the state to device arrays (any pointer may be NULL).  Asynchronous. */
int glasma_get_state_device(glasma_ctx* ctx, double* U, double* E, double* rhoA, double* rhoB);

/* ---- Differentiation form -------------------------------------------------------
 * Loss of a state (Sec. 4 energy density integrated over the layers z0 <= z < z1 of the
 * stored fields U(t), E(t - dt/2)):
 *   L = a_T^2 a_L sum_{z0 <= z < z1} [ 1/2 sum_i |E_i(x)|^2
 *                                     + sum_{i<j} 2/(a_i a_j)^2 Re Tr(1 - U_{i,j}(x)) ].
 * Gradients of L after `steps` leapfrog steps with respect to the electric field E and the
 * charges rho_A, rho_B of the starting state (links of the starting state held fixed), by
 * the reverse mode of the leapfrog step with the CPIC hop (eqs. lattice_1/2, plaquette and
 * the hop's transport rule, Sec. 3), differentiated exactly, including the derivative of
 * the matrix exponential.  The forward pass runs in the context's precision and stores a
 * checkpoint every ckpt_every steps in the caller's work buffer; the backward pass
 * recomputes each segment from its checkpoint (bitwise the forward states) and runs the
 * reverse kernels in double precision.  Reunitarisation (reunit_every) is taken as the
 * identity in the reverse pass (it moves links by rounding errors only).  The leapfrog
 * scheme only (scheme 1: GLASMA_E_ARG). */

/* Bytes of the work buffer for `steps` steps with a checkpoint every ckpt_every >= 1. */
int glasma_adjoint_layout(const glasma_params* p, int32_t steps, int32_t ckpt_every, size_t* work_bytes);

/* Advance the context `steps` steps (as glasma_step) from its current state, storing the
 * checkpoints in `work` (device, caller-owned, >= glasma_adjoint_layout bytes, kept until
 * the backward call).  Asynchronous. */
int glasma_adjoint_forward(glasma_ctx* ctx, int32_t steps, int32_t ckpt_every, void* work, size_t work_bytes);

/* Gradients of scale * L(final state) with respect to the starting state of the last
 * glasma_adjoint_forward on this context (GLASMA_E_STATE if the context stepped, was set
 * or reinitialised since, or `work` differs).  Outputs (device double arrays, each may be
 * NULL): dE0 [3][n_g][V] = dL/dE^a, drhoA0 / drhoB0 [n_g][V] = dL/drho^a at physical
 * positions, dampA / dampB [V] = sum_a base^a(x) dL/drho^a(x), the derivative with respect
 * to a per-cell amplitude of the charges (base: device [n_g][V], or NULL for the starting
 * charges themselves); L (host, may be NULL) receives the unscaled loss.  Does not change
 * the context's state.  Synchronous when L is given. */
int glasma_adjoint_backward(glasma_ctx* ctx, int32_t z0, int32_t z1, double scale, void* work, size_t work_bytes,
                            const double* baseA, const double* baseB, double* L, double* dE0, double* drhoA0,
                            double* drhoB0, double* dampA, double* dampB);

/* Reverse pass for a general loss of the final state, given its cotangent: lamU [3][n_g][V]
 * = dL/d eps^a for the left variation U_i(x) -> exp(i eps^a t^a) U_i(x) of the final links,
 * ebarE [3][n_g][V] = dL/dE^a of the final E(t - dt/2), rbarA, rbarB [n_g][V] = dL/drho^a
 * of the final charges at their physical positions (device double arrays; NULL = zero).
 * The slab energy of glasma_adjoint_backward is one such cotangent.  Outputs as there,
 * plus dU0 [3][n_g][V] (may be NULL): the same left-variation derivative for the starting
 * links.  Requirements and errors as glasma_adjoint_backward.  Asynchronous. */
int glasma_adjoint_backward_cotangent(glasma_ctx* ctx, void* work, size_t work_bytes, const double* lamU,
                                      const double* ebarE, const double* rbarA, const double* rbarB,
                                      const double* baseA, const double* baseB, double* dU0, double* dE0,
                                      double* drhoA0, double* drhoB0, double* dampA, double* dampB);

/* The loss L above at the current state (host result).  Uses the context's work buffer.
 * Synchronous. */
int glasma_slab_energy(glasma_ctx* ctx, int32_t z0, int32_t z1, double* L);

/* ---- Batched form ---------------------------------------------------------
 * Many independent events (one MV collision each) of different lattice sizes share
 * one pool of device memory and advance together: one launch per step covers every
 * event ((event, block of sites) work items), and glasma_batch_run
 * replays a captured HIP graph of `graph_chunk` steps.  The leapfrog scheme only;
 * reunitarisation (reunit_every) is fused into the step.  Each event is a regular
 * context (glasma_batch_event) for initial conditions, observables and state I/O,
 * all events must be at the same step when the batch runs. */
typedef struct glasma_batch glasma_batch;

/* Pool bytes for n_events events of sizes nz[e] x nt[e] x nt[e] with the common
 * parameters (its nz, nt are ignored; scheme must be 0). */
int glasma_batch_layout(const glasma_params* common, int32_t n_events, const int32_t* nz, const int32_t* nt,
                        size_t* pool_bytes);

/* Create the batch over a caller-owned device pool of glasma_batch_layout bytes. */
int glasma_batch_create(const glasma_params* common, int32_t n_events, const int32_t* nz, const int32_t* nt,
                        void* pool, void* stream, glasma_batch** out);

int glasma_batch_destroy(glasma_batch* b);
const char* glasma_batch_last_error(const glasma_batch* b);

/* The context of event e (owned by the batch: do not destroy it). */
int glasma_batch_event(glasma_batch* b, int32_t e, glasma_ctx** ctx);

/* Advance every event by `steps` steps; graph_chunk > 0 captures that many steps in a
 * HIP graph (kept for later calls with the same chunk and tiling) and replays it. */
int glasma_batch_run(glasma_batch* b, int32_t steps, int32_t graph_chunk);

/* N_z classes of the batch's events (distinct N_z, ascending): n_classes, and, for each
 * class k, nz_of_class[k] and events_of_class[k] (either array may be NULL; each needs room
 * for n_events entries at most).  Host values. */
int glasma_batch_classes(const glasma_batch* b, int32_t* n_classes, int32_t* nz_of_class, int32_t* events_of_class);

/* Event average of T^{mu nu}(z) at the current integer time (Sec. 2 eq. ev: the average
 * over the MV ensemble, estimated by the mean over the batch's independent events; Sec. 4
 * <T^{mu nu}>).  Every event's observables (as glasma_observe, into the pool), then, on the
 * device, the eps, p_L, p_T, S_L slices averaged
 *   class_avg: per N_z class (order of glasma_batch_classes), the mean over that class's
 *              events of the [4][N_z] slices, the classes' blocks one after another;
 *   grid_avg:  [4][n_grid], the mean over all events on a common grid of relative position
 *              z / N_z: bin b of an event is the mean of its layers z with
 *              floor(z n_grid / N_z) = b (1 <= n_grid <= the smallest N_z, so no bin is
 *              empty);
 *   per_event: (may be NULL) every event's observables buffer, 4 N_z + GLASMA_OBS_NSCALARS
 *              doubles each, events in order.
 * All output pointers are caller-owned device double arrays.  Asynchronous on the batch's
 * stream; GLASMA_E_ARG for a bad n_grid or NULL outputs, GLASMA_E_STATE if an event has
 * no state. */
int glasma_batch_observe(glasma_batch* b, int32_t n_grid, double* class_avg, double* grid_avg, double* per_event);

/* Work-item tiling: sites per item (64, 128 or 256 threads per workgroup) and the
 * number of persistent workgroups that loop over the items, or 0: one workgroup per item,
 * a kernel without the loop (for FP32 it fits four waves per SIMD, the looping one three). */
int glasma_batch_set_tiling(glasma_batch* b, int32_t sites_per_item, int32_t grid);

/* Autotuner: times every tiling candidate (12: sites per item 64, 128, 256 x grid 0, 4096,
 * 2048, 1024) over `steps` steps (HIP events, after one untimed step of that candidate)
 * and keeps the fastest; writes a JSON report (may be NULL).  Advances the state by
 * 13 * steps + 12 steps, so call it before setting up the events that are to be measured. */
int glasma_batch_autotune(glasma_batch* b, int32_t steps, char* report, size_t report_len);

/* Host-side evaluation of the library's group kernels, for CPU tests of the
 * device algebra (the same inline functions the GPU kernels use).  op:
 *   0: out = exp(i s X) as a link      in = [s, X^a]                (n_g + 1 in)
 *   1: out = -i Log(W) components      in = W link reals             (r_U in)
 *   2: out = P(M) components           in = M link reals             (r_U in)
 *   3: out = U^dag X U components      in = [U link reals, X^a]      (r_U + n_g in)
 *   4: out = reunitarised link         in = link reals
 *   5: out = [unitarity violation]     in = link reals
 *   6: out = A B (link)                in = [A, B] link reals
 *   7: out = c int_0^1 exp(-i s c X) L exp(i s c X) ds components, in = [c, X^a, L^a]
 *        (1 + 2 n_g in; the transpose of the derivative of exp(i c X), double arithmetic)
 * fp = 64 or 32 selects the arithmetic.  n items are processed; in/out are packed
 * item after item.  Returns GLASMA_E_ARG for an unknown op. */
int glasma_host_group_op(int32_t nc, int32_t fp, int32_t op, int64_t n, const double* in, double* out);

#ifdef __cplusplus
}
#endif
#endif /* GLASMA_H */
