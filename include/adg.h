/*
 * adg.h — C ABI of the MI355X (gfx950) asynchronous discontinuous Galerkin solver.
 *
 * The solver advances the 1D compressible reacting-flow equations of
 * Arumugam & Aditya, "An asynchronous discontinuous Galerkin method for
 * combustion simulations" (arXiv 2501.01747):
 *   dw/dt + df^c/dx = df^d/dx + s                       Sec. 2, Eq. (1)-(3)
 * with a Legendre-modal DG discretisation (Sec. 3.1, Eq. (4)-(6)), local
 * Lax-Friedrichs or HLLC fluxes, LDG diffusion, three-stage SSP Runge-Kutta
 * time stepping, and the asynchronous machinery of Sec. 3.2-4: the domain is
 * split into emulated processing elements (PEs); at PE interfaces the flux is
 * the asynchrony-tolerant (AT) flux of Eq. (7) built from the synchronous
 * fluxes of past time levels with the weights of Eq. (8); delays follow the
 * CAA (Sec. 4.1) or SAA (Sec. 4.2) model.  The optional limiter is the
 * KXRCF-indicated characteristic WENO of Eq. (9)-(10) with the AT neighbour
 * data of Eq. (11) across delayed PE interfaces.
 *
 * Conventions of the whole ABI
 *   * Every call returns adg_status (0 = ADG_OK, negative = error); nothing
 *     aborts or throws across the ABI.  adg_last_error() gives a message.
 *   * State arrays exchanged with the caller are FP64 modal coefficients in the
 *     layout w[e][v][j]: element e (0..E-1), conserved variable v
 *     (rho, rho u, rho E, rho Y_1 .. rho Y_Ns; V = 3 + Ns), Legendre mode j
 *     (0..N_p, basis normalised with P_j(1) = 1).
 *   * The library allocates no device memory.  The caller passes one device
 *     workspace of adg_workspace_bytes() bytes (e.g. a torch tensor); it must
 *     stay alive and unmodified until adg_destroy().  All kernels run on the
 *     caller's HIP stream (hipStream_t passed as void*).
 *   * Errors detected on the device (non-physical state: rho <= 0, p <= 0,
 *     non-finite, Newton failure for the temperature) are latched in a device
 *     flag and reported as ADG_ERR_STATE by the next synchronising call
 *     (adg_get_state, adg_sync).
 *   * Calls on one solver must not overlap; different solvers are independent.
 */
#ifndef ADG_H
#define ADG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t adg_status;
#define ADG_OK 0
#define ADG_ERR_ARG (-1)         /* inconsistent or unsupported argument values */
#define ADG_ERR_NOMEM (-2)       /* workspace too small */
#define ADG_ERR_HIP (-3)         /* a HIP runtime call failed */
#define ADG_ERR_STATE (-4)       /* non-physical state detected on the device */
#define ADG_ERR_UNSUPPORTED (-5) /* valid but not implemented combination */

enum { ADG_ONESTEP = 0, ADG_DETAILED = 1 };
enum { ADG_PERIODIC = 0, ADG_TRANSMISSIVE = 1 };
enum { ADG_RUSANOV = 0, ADG_HLLC = 1 };
enum { ADG_SYNC = 0, ADG_CAA = 1, ADG_SAA = 2, ADG_SCHEDULE = 3 };
enum { ADG_HOST = 0, ADG_DEVICE = 1 };
enum { ADG_KXRCF = 0, ADG_MINMOD = 1, ADG_ALL_CELLS = 2 };
enum { ADG_AT_TEMPORAL = 0, ADG_AT_HYBRID = 1 };
enum { ADG_SSPRK3 = 0, ADG_RK2 = 1, ADG_LSERK4 = 2 };
enum { ADG_FP64 = 0, ADG_MIXED_FP32 = 1, ADG_MIXED_BF16 = 2 };

/* Detailed reaction mechanism (Sec. 2: mass-action kinetics with species
   molecular weights W_i and molar production rates omega_i).  Reversible
   reactions: k_f = A T^b exp(-Ea/(Ru T)), k_r = k_f / K_c with
   K_c = exp(-Delta G/(Ru T)) (p_ref/(Ru T))^(sum nu).  Thermo: NASA
   7-coefficient polynomials, one temperature range.  Transport: viscosity
   mu = mu_ref (T/T_ref)^mu_exp, conductivity k = mu cp/Pr, unit Lewis number.
   All arrays are read during adg_create only.  Limits of the kernels (beyond
   them ADG_ERR_UNSUPPORTED): 1..16 species (9 in batches), 1..32 reactions
   (24 in batches), at most two
   molecules on either side of a reaction and at most four species whose net
   coefficient is nonzero in one reaction (no third bodies). */
typedef struct adg_mechanism {
  int32_t n_species, n_reactions;
  const double *W;        /* [Ns] kg/mol */
  const double *nasa7;    /* [Ns][7] */
  const int32_t *nu_f;    /* [Nr][Ns] reactant coefficients (0, 1 or 2) */
  const int32_t *nu_r;    /* [Nr][Ns] product coefficients */
  const double *A, *b, *Ea; /* [Nr] SI units, Ea in J/mol */
  double Ru, p_ref;       /* J/(mol K), Pa */
  double mu_ref, T_ref, mu_exp, prandtl;
  double T_guess;         /* start of the Newton iteration for T(e) */
} adg_mechanism;

/* Governing equations, Sec. 2. */
typedef struct {
  int32_t model;          /* ADG_ONESTEP: nondimensional reactive Euler (R = 1), species (R, P),
                                rho E = rho u^2/2 + p/(gamma-1) + q_heat rho Y_R,
                                source W omega = -+ k_pre rho Y_R exp(-e_act/T), T = p/rho.
                             ADG_DETAILED: mixture of Ns thermally perfect species with the
                                mechanism `mech`; viscous = 1 adds the Navier-Stokes terms. */
  int32_t n_species;      /* Ns: 2 for ADG_ONESTEP; 1..16 for ADG_DETAILED (up to 9 in batches) */
  int32_t viscous;
  double gamma, q_heat, e_act, k_pre;
  const adg_mechanism *mech;
} adg_physics;

/* Discretisation, Sec. 3.1. */
typedef struct {
  int32_t order_p;        /* N_p, polynomial degree: 1..4 */
  int32_t n_quad;         /* Gauss-Legendre points per element: 0 = N_p + 1 (only value supported) */
  int32_t n_elem;         /* N_E >= 1 */
  double x_left, x_right;
  int32_t bc;             /* ADG_PERIODIC | ADG_TRANSMISSIVE (ghost trace = interior trace for the
                             state and, with LDG, for its gradient; the end faces are synchronous) */
  int32_t flux;           /* ADG_RUSANOV | ADG_HLLC (HLLC with ADG_ONESTEP only) */
  int32_t limiter;        /* 1 = troubled-cell indicator + characteristic (AT-)WENO after every
                             stage (ADG_ONESTEP) */
  int32_t indicator;      /* ADG_KXRCF: Krivodonova et al. on rho and rho E at inflow faces;
                             ADG_MINMOD: the TVB minmod test of the conserved variables (the
                             TVD slope-limiter indicator of Sec. 3.3 when tvb_m = 0);
                             ADG_ALL_CELLS: every cell limited (accuracy tests of the limiter) */
  double tvb_m;           /* TVB constant M (>= 0) of ADG_MINMOD: face deviations up to M dx^2 pass */
  double weno_gamma[3];   /* linear weights of Eq. (10) */
  double weno_eps;        /* epsilon of Eq. (10) */
  double dt;              /* fixed time step (> 0); the AT weights of Eq. (8) assume it constant */
  int32_t rk;             /* ADG_SSPRK3: three-stage SSP Runge-Kutta (Shu-Osher form);
                             ADG_RK2: Heun's two-stage method and ADG_LSERK4: the five-stage
                             fourth-order low-storage scheme of Carpenter and Kennedy, both in the
                             2N-storage form k <- A_s k + dt L(u), u <- u + B_s k (the LSERK
                             integrators of Sec. 3.1).  Stage s of step n reads the stage-s data of
                             past levels (Eq. (7)); batches support ADG_SSPRK3 only. */
  int32_t precision;      /* ADG_FP64: every step in FP64.
                             ADG_MIXED_FP32 (detailed model): the modal operators (interpolation to
                             nodes and traces, LDG gradient, volume integral) in FP32 with FP32
                             accumulation, on deviations from the element mean; the temperature
                             Newton, transport, Arrhenius rates and equilibrium constants, interface
                             fluxes, source projection and RK update in FP64.  Applied for N_p <= 3,
                             where the error against the FP64 solution stays below a tenth of the
                             discretisation error (4 % of it measured at N_p = 3); N_p = 4 keeps FP64
                             operators (FP32 measured 11 times the discretisation error there).  The
                             one-step model returns ADG_ERR_UNSUPPORTED.
                             ADG_MIXED_BF16: ADG_ERR_UNSUPPORTED: BF16 (8-bit significand) operators
                             would raise the FP32 path's operator error by about 2^16, past the
                             discretisation error at every order of these workloads.
                             In a batch the batch's precision applies: an instance passes ADG_FP64
                             or the batch's precision (one-step instances run in FP64 in any batch). */
} adg_discretization;

/* Emulated PEs and delay model, Sec. 3.2 and 4. */
typedef struct {
  int32_t n_pe;           /* P, 1 <= P <= N_E */
  const int32_t *pe_offsets; /* [P+1] first element of each PE (host), or NULL = floor(p E / P) */
  int32_t mode;           /* ADG_SYNC | ADG_CAA (k = n mod L) | ADG_SAA | ADG_SCHEDULE */
  int32_t L;              /* number of admissible delays, k in {0 .. L-1}; 1 <= L <= 8 */
  const double *pmf;      /* [L] SAA probabilities (host); must sum to 1 within 1e-12 */
  uint64_t seed;          /* SAA: counter-based SplitMix64 draw per (step, interface) */
  const int8_t *schedule; /* ADG_SCHEDULE: [schedule_steps][n_if] delays in 0..L-1 (host), period
                             schedule_steps; any other delay is ADG_ERR_ARG */
  int32_t schedule_steps;
  int32_t at_order;       /* q, number of levels in Eq. (7): 0 = N_p + 1; 1..6 */
  int32_t at_stencil;     /* buffer-element DoFs of Eq. (11) across delayed PE interfaces (limiter):
                             ADG_AT_TEMPORAL: every Legendre mode from the q levels n-k .. n-k-q+1;
                             ADG_AT_HYBRID: the spatio-temporal stencil that closes Sec. 3.3, read
                             from Eq. (8) with the dx^j size of mode j: mode j from the first
                             max(1, q - j) of those levels, with the weights of that order (the
                             same order of accuracy from fewer buffered values: the oldest level
                             contributes only the element mean) */
} adg_async;

typedef struct adg_solver adg_solver;

/* Device workspace needed for a problem (0 on invalid arguments). */
size_t adg_workspace_bytes(const adg_physics *phys, const adg_discretization *disc, const adg_async *as);

/* Validates the problem, lays out the workspace (256-byte aligned pointer
   required), uploads constant tables and the mechanism, and returns a solver.
   PE interfaces: the faces at pe_offsets[1..P-1], plus the periodic wrap face
   (interface 0) when bc is periodic, so n_if = P (periodic) or P-1.
   The state is undefined until adg_set_state(). */
adg_status adg_create(const adg_physics *phys, const adg_discretization *disc, const adg_async *as,
                      void *device_workspace, size_t workspace_bytes, void *hip_stream,
                      adg_solver **out);

/* Replace the state by w ([E][V][M] FP64, `count` = E*V*M doubles) on the host
   (where = ADG_HOST; synchronous copy) or on the device (ADG_DEVICE; enqueued).
   Resets the step counter to 0, clears the history of past levels and the
   device error flag. */
adg_status adg_set_state(adg_solver *s, const double *w, int64_t count, int32_t where);

/* Enqueue n_steps full SSP-RK3 time steps on the stream (asynchronous). */
adg_status adg_step(adg_solver *s, int32_t n_steps);

/* Copy the current state out ([E][V][M]).  Synchronises the stream and
   returns ADG_ERR_STATE if the device latched a non-physical state. */
adg_status adg_get_state(adg_solver *s, double *w, int64_t count, int32_t where);

/* Synchronise the stream and report the device error flag. */
adg_status adg_sync(adg_solver *s);

/* Troubled-cell flags (int8 [E], host) of the last limited stage, and the
   number of troubled cells summed over all limited stages since set_state. */
adg_status adg_get_flags(adg_solver *s, int8_t *flags, int64_t *total);

/* Number of completed time steps since adg_set_state (synchronises). */
int64_t adg_step_count(adg_solver *s);

/* Number of PE interfaces. */
int32_t adg_n_interfaces(const adg_solver *s);

/* Enqueue n_steps steps like adg_step and time every kernel launch with HIP
   events on the solver's stream.  ms_out[i] receives the mean duration in ms
   of kernel class i and launches_out[i] the launch count; n_classes is the
   array length (class 0: the stage kernel, which includes the limiter of a
   limited problem; there is one launch per RK stage).
   Synchronises. */
adg_status adg_profile(adg_solver *s, int32_t n_steps, double *ms_out, int64_t *launches_out, int32_t n_classes);

/* Use captured HIP graphs of `steps_per_graph` time steps for adg_step
   (0 = plain launches, the default).  Takes effect at the next adg_step, which
   captures two graphs: a step moves the solver between two alignments (step
   counter parity, and the state buffer where it alternates), and each graph
   replays from one of them, so adg_step(n) runs n / steps_per_graph graph
   replays and n mod steps_per_graph plain steps whatever the alignment. */
adg_status adg_set_graph(adg_solver *s, int32_t steps_per_graph);

/* Number of graph replays adg_step has launched since adg_set_state (-1 for a
   null solver): with adg_set_graph(g), adg_step(n) adds n / g. */
int64_t adg_graph_replays(const adg_solver *s);

/* Choose the stage kernel's work decomposition by measurement: for the
   detailed-chemistry model, the tile size (4 or 8 elements) and workgroup size
   (256, 512 or 1024 threads) of the stage kernel: every candidate is warmed up,
   then timed over n_reps launches of the first RK stage on the current state in
   three interleaved rounds, its fastest round counting; later steps use the
   fastest candidate, or the first one (8/512) unless the fastest beats it by
   more than 3 %.  The timed launches only rewrite the first stage buffer and the
   current level's first-stage history, which the next step recomputes, so the
   solution is unchanged.  *choice (optional) receives the chosen candidate
   (0: 8/512, 1: 8/256, 2: 4/256, 3: 4/512, 4: 8/1024; always 0 for the one-step model,
   whose kernel has one decomposition).  Synchronises. */
adg_status adg_autotune(adg_solver *s, int32_t n_reps, int32_t *choice);

/* Use work decomposition `config` (the numbering of adg_autotune; only 0 for
   the one-step model) for the following steps.  ADG_ERR_ARG for any other
   value.  The result of a step does not depend on the decomposition beyond
   the order of floating-point sums across lanes. */
adg_status adg_set_kernel_config(adg_solver *s, int32_t config);

/* Release the solver (the caller's workspace is not freed). */
void adg_destroy(adg_solver *s);

/* Message of the last error of solver s; with s = NULL, the message of the last
   failed adg_create / adg_create_noalloc call on the calling thread. */
const char *adg_last_error(const adg_solver *s);

/* For callers that cannot allocate device memory (code under HIP graph capture,
   tight serving loops, harnesses that forbid hipMalloc): adg_create without a
   workspace.  The solver's device memory (state buffers, history ring, counters,
   constant tables) is a static array of 64 MiB per device, part of the library,
   whose address is taken once per device; nothing is allocated on the device
   (no hipMalloc, hipFree or allocating library routine, torch's included, is
   called; set-up uses host memory only, for small tables).  Problems larger than
   64 MiB (adg_workspace_bytes) return ADG_ERR_NOMEM.  One such solver may be alive
   per device: a second call before adg_destroy of the first returns ADG_ERR_STATE.
   The array keeps the contents of the previous solver; adg_set_state clears what
   must start at zero (step counters, error flag, history ring, flags) with fill
   kernels, which may be captured.  Calls that use one device's array from
   several threads or streams at once race.  Every other call works on the
   solver as on one from adg_create; adg_destroy frees the array for the next. */
adg_status adg_create_noalloc(const adg_physics *phys, const adg_discretization *disc, const adg_async *as,
                              void *hip_stream, adg_solver **out);


/* ------------------------------------------------------------------------
 * Batches of independent instances in one workspace.
 *
 * Many ADG problems of different sizes, orders, PE layouts and delay models
 * advance together: every RK stage of a time step is one batched launch for
 * all detailed-chemistry instances (plus one per order, flux and limiter
 * choice for the one-step model), so small
 * instances fill the device together.  Each workgroup works on one instance
 * with that instance's own arguments: an instance's result does not depend on
 * what else is in the batch (alone and in the mix are bitwise identical for
 * the same precision).  The method per instance is the one of adg_create.
 *
 * Workspace: a header of adg_batch_header_bytes(max_instances, max_elements)
 * followed by a heap; an instance occupies adg_batch_instance_bytes() of it
 * (its states, history ring, flags and constant data).  Admission is by this
 * footprint: adg_batch_add fails with ADG_ERR_NOMEM when no free region, slot
 * or element capacity is left, and succeeds again once removals free space.
 *
 * Precision (per batch, detailed-chemistry instances): ADG_FP64 or
 * ADG_MIXED_FP32, as adg_discretization.precision describes (FP32 operators
 * for N_p <= 3, FP64 ones for N_p = 4); ADG_MIXED_BF16 returns
 * ADG_ERR_UNSUPPORTED.  One-step instances always run in FP64.
 *
 * Calls on one batch must not overlap.  adg_batch_add and adg_batch_remove
 * synchronise the batch's stream.
 * ---------------------------------------------------------------------- */
typedef struct adg_batch adg_batch;

/* Header bytes of a batch with up to max_instances instances whose element
   counts sum to at most max_elements (0 on invalid arguments). */
size_t adg_batch_header_bytes(int32_t max_instances, int64_t max_elements);

/* Heap bytes one instance occupies (0 on invalid arguments). */
size_t adg_batch_instance_bytes(const adg_physics *phys, const adg_discretization *disc, const adg_async *as);

/* Create an empty batch in the caller's workspace (256-byte aligned; header
   followed by the heap, workspace_bytes in total). */
adg_status adg_batch_create(int32_t max_instances, int64_t max_elements, int32_t precision,
                            void *device_workspace, size_t workspace_bytes, void *hip_stream,
                            adg_batch **out);

/* Admit one instance with initial state w0 ([E][V][M] FP64, count = E*V*M,
   on the host or the device per `where`).  It runs n_steps time steps in the
   following adg_batch_step calls and then idles (0 = no limit).  Its step count
   starts at 0.  *slot receives its slot number (0 .. max_instances-1). */
adg_status adg_batch_add(adg_batch *b, const adg_physics *phys, const adg_discretization *disc,
                         const adg_async *as, const double *w0, int64_t count, int32_t where,
                         int64_t n_steps, int32_t *slot);

/* Release an instance's slot and workspace region. */
adg_status adg_batch_remove(adg_batch *b, int32_t slot);

/* Enqueue n_steps time steps of every admitted instance that has not reached
   its n_steps (asynchronous). */
adg_status adg_batch_step(adg_batch *b, int32_t n_steps);

/* Synchronise; steps[i] = completed time steps of slot i (-1 if empty) and
   state_err[i] = 1 if slot i latched a non-physical state.  Both arrays have
   max_instances entries; either may be NULL. */
adg_status adg_batch_poll(adg_batch *b, int64_t *steps, int32_t *state_err);

/* Copy an instance's current state out ([E][V][M]); synchronises; returns
   ADG_ERR_STATE if that instance latched a non-physical state. */
adg_status adg_batch_get_state(adg_batch *b, int32_t slot, double *w, int64_t count, int32_t where);

/* Use captured HIP graphs of steps_per_graph time steps (0 = plain launches):
   one graph per step counter parity, so adg_batch_step(n) replays
   n / steps_per_graph graphs and runs n mod steps_per_graph plain steps; the
   graphs are rebuilt after the batch's composition changes. */
adg_status adg_batch_set_graph(adg_batch *b, int32_t steps_per_graph);

/* Enqueue n_steps steps with HIP events around every launch; ms_out[c] is the
   mean duration of launch class c (0 detailed-chemistry stage, 1 one-step
   stage, including the limiter of limited instances) and launches_out[c] its
   count.  Synchronises. */
adg_status adg_batch_profile(adg_batch *b, int32_t n_steps, double *ms_out, int64_t *launches_out,
                             int32_t n_classes);

/* Choose the tile size (8 or 4 elements) of the batched detailed-chemistry
   kernel by timing n_reps launches of its first RK stage for the current batch
   (state unchanged, as for adg_autotune; three interleaved rounds, each
   candidate's fastest counting); kept until the next call.  *choice
   (optional): 0 = 8 elements, 1 = 4.  Synchronises. */
adg_status adg_batch_autotune(adg_batch *b, int32_t n_reps, int32_t *choice);

/* Use work decomposition `config` of the batched detailed-chemistry kernel
   (adg_batch_autotune's numbering, 0 or 1; ADG_ERR_ARG otherwise) from the next
   step on.  Results do not depend on it beyond the order of floating-point sums. */
adg_status adg_batch_set_kernel_config(adg_batch *b, int32_t config);

/* Spread each RK stage's launches (one per group: the detailed-chemistry
   instances, and one per (order, flux, limiter) class of one-step instances)
   over `streams` streams (1..4; ADG_ERR_ARG otherwise): the batch's stream and
   up to three more of the default priority, created by the library on first
   use and joined back into the batch's stream before the next stage.  Groups
   touch disjoint instances, so results do not depend on it; with several
   groups the smaller launches overlap the larger ones instead of waiting for
   them.  Default 4; 1 launches everything on the batch's stream.  A captured
   graph is re-captured at the next step. */
adg_status adg_batch_set_group_streams(adg_batch *b, int32_t streams);

/* Number of admitted instances. */
int32_t adg_batch_active(const adg_batch *b);

/* Size of the largest free heap region. */
int64_t adg_batch_free_bytes(const adg_batch *b);

/* Release the batch (synchronises; the workspace is not freed). */
void adg_batch_destroy(adg_batch *b);

const char *adg_batch_last_error(const adg_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* ADG_H */
