/*
 * felbm.h — C ABI of the MI355X (gfx950) finite element lattice Boltzmann
 * step for two-phase flow with wetting walls (Matin, Misztal,
 * Hernandez-Garcia, Mathiesen, "Finite Element Lattice Boltzmann Simulations
 * of Contact Line Dynamics", arXiv:1708.04678).
 *
 * One time step (Sec. II.C-D) on a P1 triangle mesh with D2Q9 populations
 * g (pressure/momentum) and h (composition), 18 values per node:
 *   moments C, p, u (eq:velocity, eq:pressure) -> element gradients ->
 *   nodal patch Laplacian of C with the wetting flux (eqn:lapl_int_mp,
 *   eq. bc2) -> chemical potential (eqn:mp_mu) -> element Laplacian of mu
 *   -> P0 element forces (eq:G, eq:H, eq:intF) -> BGK collision
 *   (eqn::collide) -> Galerkin streaming right-hand side (eqn::stream,
 *   eq:galerkin_lbm) -> consistent-mass solve with the lumped-mass
 *   preconditioner -> wall operator.
 *
 * Conventions for every function below:
 *   - return value: FELBM_OK (0) or a negative FELBM_E* code; nothing throws
 *     across the ABI; felbm_last_error() gives a message owned by the
 *     context, valid until the next call on that context.
 *   - host arrays are owned by the caller and copied; device memory is owned
 *     by the library.  Arrays are in the caller's node / triangle order.
 *   - floating point host arrays are double; integer arrays int32.
 *   - all validation happens on the host before any device work.
 *   - one context per host thread; calls on one context are not thread safe.
 *   - results are deterministic: no atomics, fixed reduction orders.
 */
#ifndef FELBM_H
#define FELBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  FELBM_OK = 0,
  FELBM_EINVAL = -1,     /* null pointer, bad size or bad parameter            */
  FELBM_EMESH = -2,      /* index out of range, non-positive unwrapped area,
                            non-manifold edge, boundary edge that is neither a
                            wall nor periodic, wall edge not on the boundary   */
  FELBM_ESTATE = -3,     /* call out of order (e.g. step before init)          */
  FELBM_ENONFINITE = -4, /* a NaN / Inf appeared in the state                  */
  FELBM_ESOLVER = -5,    /* solver configuration rejected                      */
  FELBM_EDEVICE = -6,    /* HIP runtime error                                  */
  FELBM_ENOMEM = -7      /* device allocation failed                           */
};

enum { FELBM_FP64 = 0, FELBM_FP32 = 1 };

/* Physical and numerical parameters (Sec. II and II.A).
 *   sigma, xi      surface tension and interface width; the free energy
 *                  constants follow from xi = sqrt(8 kappa/beta) and
 *                  sigma = sqrt(2 kappa beta)/6 (Sec. II, after eqn:mp_mu)
 *   mobility       M of eqn:mp_che
 *   rho_l, rho_v   phase densities, rho = C rho_l + (1 - C) rho_v
 *   nu_l, nu_v     kinematic viscosities; tau = nu / (c_s^2 dt) per phase and
 *                  1/tau = C/tau_l + (1 - C)/tau_v (Sec. II.A)
 *   dt             time step
 *   precision      FELBM_FP64: everything in double.  FELBM_FP32: populations,
 *                  velocity/pressure fields, forces, streaming and solve in
 *                  float; the chain C -> lap C -> mu -> grad mu -> lap mu,
 *                  all global reductions and the conserved composition in
 *                  double: C = sum_a h_a + r with a per-node FP64 remainder r,
 *                  whose increment is the FP64 zeroth h-moment of the
 *                  streaming right-hand side solved by the same sweeps with
 *                  exactly mass-preserving column sums.
 *   solver_sweeps  K >= 0: the mass-matrix system M11 x = b is solved by K
 *                  preconditioned Richardson sweeps from x0 = b/m whose step
 *                  lengths are the reciprocal Chebyshev roots for the spectrum
 *                  bounds below, i.e. the degree-K Chebyshev iterate with the
 *                  lumped-mass preconditioner (error <= 2/T_K((b+a)/(b-a))).
 *                  K = 0 is the lumped-mass solve.  Every sweep preserves
 *                  sum_i m_i x_i = sum_i b_i, hence mass.
 *   lambda_min/max bounds of the spectrum of diag(m)^-1 M11; 0/0 selects the
 *                  bounds [1/4, 1] that hold for every P1 triangle mesh.
 *   kernels        FELBM_KERNELS_AUTO: the right-hand side and the sweeps run
 *                  on LDS-staged 256-node tiles whenever every tile's halo
 *                  has at most 128 nodes and every mass-matrix row at most 12
 *                  off-diagonal entries (otherwise the global-gather kernels);
 *                  FELBM_KERNELS_GLOBAL: always the global-gather kernels
 *                  (same arithmetic, for meshes and tests that need them).
 *   force_scheme   FELBM_FORCES_MIXED: the paper's scheme, forces constant per
 *                  element at the barycentric field values (Sec. II.C,
 *                  eq:intF).  FELBM_FORCES_NODAL: the comparison scheme of the
 *                  parasitic-current table (Sec. III.A), forces as P1 fields
 *                  from nodal values and area-weighted nodal gradients, nodal
 *                  lap mu by the vertex-patch operator with zero wall flux;
 *                  FP64 only, no adjoint.  FELBM_FORCES_NODAL_COLLIDE: the
 *                  same nodal forces integrated locally in the collision step
 *                  (the authors' earlier scheme, Sec. II.C): trapezoid rule on
 *                  the force, psi_bar = psi + dt/2 (Omega - F), collision
 *                  psi_hat = psi_bar - (psi_bar - psi_eq + dt/2 F)/(tau + 1/2)
 *                  + dt F, streaming without force; the velocity and pressure
 *                  carry half the force's moments (rho u += dt/2 mu grad C,
 *                  p += dt/2 c_s^2 u . grad rho), the h equilibrium uses
 *                  C + dt/2 M lap mu, wall nodes are at rest, and felbm_init
 *                  sets psi_bar = psi_eq - dt/2 F.  FP64 only, no adjoint, not
 *                  for felbm_diagnostics_noalloc.                            */
enum { FELBM_KERNELS_AUTO = 0, FELBM_KERNELS_GLOBAL = 1 };
enum { FELBM_FORCES_MIXED = 0, FELBM_FORCES_NODAL = 1, FELBM_FORCES_NODAL_COLLIDE = 2 };

typedef struct {
  double sigma, xi, mobility;
  double rho_l, rho_v, nu_l, nu_v, dt;
  int32_t precision;
  int32_t solver_sweeps;
  double lambda_min, lambda_max;
  int32_t kernels;
  int32_t force_scheme;
} felbm_params;

/* Global FP64 reductions of the current state (Sec. III) and the state of
 * the mass-matrix solve (end of Sec. II.C).
 *   mass     sum_i m_i C_i with m the lumped mass vector (int C dx)
 *   mean_ke  <T> = 0.5 sum_i rho_i |u_i|^2 / N (caption of the mobility figure)
 *   max_u    max_i |u_i|
 *   band_ke  mean of rho |u|^2 over nodes in the band set by felbm_set_band
 *            (the <rho u.u> of the parasitic-current table); 0 if unset
 *   band_nodes number of nodes in that band
 *   nonfinite 1 if any population is NaN/Inf
 *   solver_sweeps    K, the fixed number of preconditioned sweeps per step
 *   solver_residual  relative residual of the most recently sampled solve
 *                    (see felbm_set_residual_sampling): the largest over the
 *                    18 systems of ||M11 x_K - b|| / ||b|| in the norm
 *                    ||v||^2 = sum_i v_i^2 / m_i; -1 if none was sampled
 *   residual_step    the step whose solve was sampled; -1 if none
 * felbm_history fills the first eight members only (solver_* = 0 / -1).  */
typedef struct {
  int64_t step;
  double mass, mean_ke, max_u, band_ke;
  int64_t band_nodes;
  int32_t nonfinite;
  int32_t solver_sweeps;
  double solver_residual;
  int64_t residual_step;
} felbm_diag;

/* Fields for felbm_read.  Nodal fields have N values, element fields E. */
enum {
  FELBM_FIELD_C = 0,     /* composition sum_a h_a                       (N) */
  FELBM_FIELD_RHO = 1,   /* density                                      (N) */
  FELBM_FIELD_P = 2,     /* pressure sum_a g_a                           (N) */
  FELBM_FIELD_UX = 3,    /* velocity (1/(c_s^2 rho)) sum_a e_a g_a       (N) */
  FELBM_FIELD_UY = 4,
  FELBM_FIELD_MU = 5,    /* chemical potential                           (N) */
  FELBM_FIELD_LAPC = 6,  /* nodal patch Laplacian of C                   (N) */
  FELBM_FIELD_LAPMU = 7  /* element Laplacian of mu                      (E) */
};

typedef struct felbm_ctx felbm_ctx;

/* Create a context on the current HIP device.  params is copied.
 * Errors: EINVAL (null, non-positive dt/xi/densities/viscosities, negative
 * sigma or mobility, bad precision, solver_sweeps < 0 or > 256,
 * 0 < lambda_min < lambda_max violated), EDEVICE, ENOMEM. */
int felbm_create(const felbm_params* params, felbm_ctx** out);

/* Message for the last failed call on ctx (or on creation when ctx is NULL). */
const char* felbm_last_error(const felbm_ctx* ctx);

/* Upload an unstructured P1 triangle mesh (Sec. II.C: nodal unknowns,
 * piecewise-linear shape functions).
 *   xy         [n_nodes][2] node coordinates
 *   tri        [n_tris][3] vertex indices, counter-clockwise after the x
 *              unwrap (minimum image when period_x > 0)
 *   wall_edge  [n_wall_edges][2] node pairs of solid-wall boundary edges;
 *              every boundary edge must be listed, and only those
 *   period_x   > 0: x is periodic with this period (nodes on the seam are
 *              shared by the elements on both sides); 0: not periodic
 * Builds element geometry in FP64, element adjacency, the node->element
 * gather lists and the consistent mass matrix on the host, then copies them
 * to the device.  May be called once per context.
 * Errors: EINVAL, EMESH, ESTATE (second call), ENOMEM, EDEVICE. */
int felbm_upload_mesh(felbm_ctx* ctx, int64_t n_nodes, const double* xy, int64_t n_tris,
                      const int32_t* tri, int64_t n_wall_edges, const int32_t* wall_edge,
                      double period_x);

/* Per-node wetting potential Omega_c (Young: cos theta = -Omega_c, Sec. II.B),
 * [n_nodes], read at wall nodes only; the wall flux uses
 * phi_c / kappa = Omega_c sqrt(2 kappa beta) / kappa in eq. bc2.
 * Defaults to 0 (neutral wall).  Errors: EINVAL (null, non-finite, or
 * nonzero with kappa = 0), ESTATE (no mesh). */
int felbm_set_wetting(felbm_ctx* ctx, const double* omega_c);

/* The same with omega_c_dev [n_nodes] in device memory (caller node order,
 * double), for callers whose data already lives on the GPU (an autograd
 * graph).  The values are checked on the device first, so a rejected call
 * leaves the wetting field as it was; the bound stream is synchronised
 * before returning, after which omega_c_dev may be reused.  Same errors as
 * felbm_set_wetting, plus EDEVICE. */
int felbm_set_wetting_device(felbm_ctx* ctx, const double* omega_c_dev);

/* Initialise the populations to the equilibria (eqn::g_eq, eqn::f_eq) of
 * C [n_nodes], u [n_nodes][2] (NULL = 0) and p [n_nodes] (NULL = 0), then
 * apply the wall operator.  Resets the step counter.
 * Errors: EINVAL (null C, non-finite value), ESTATE (no mesh). */
int felbm_init(felbm_ctx* ctx, const double* C, const double* u, const double* p);

/* Advance n_steps >= 0 time steps on the bound stream and wait for them.
 * Errors: ESTATE (not initialised), ENONFINITE (the per-step FP64 check saw
 * a NaN/Inf; felbm_last_error names the first such step), EDEVICE. */
int felbm_step(felbm_ctx* ctx, int64_t n_steps);

/* Same as felbm_step without waiting and without the non-finite check:
 * work is queued on the bound stream.  For timing loops. */
int felbm_step_async(felbm_ctx* ctx, int64_t n_steps);

/* Copy a field derived from the current state to out (caller-owned double,
 * N or E values as listed above).  Errors: EINVAL, ESTATE. */
int felbm_read(felbm_ctx* ctx, int32_t field, double* out);

/* A nodal field (FELBM_FIELD_C .. FELBM_FIELD_LAPC) written to out_dev
 * [n_nodes] in device memory (caller-owned, caller node order, double), with
 * the same values as felbm_read.  Queued on the bound stream without
 * waiting: work the caller queues after it on that stream sees the values.
 * Errors: EINVAL (null, element field), ESTATE, EDEVICE. */
int felbm_read_device(felbm_ctx* ctx, int32_t field, double* out_dev);

/* Copy the current populations to out [18][n_nodes] (g_0..g_8, h_0..h_8) as
 * double.  In FELBM_FP32 the composition is sum_a h_a plus an FP64 remainder
 * (see felbm_params.precision), so FELBM_FIELD_C is the exact composition.
 * Errors: EINVAL, ESTATE. */
int felbm_read_populations(felbm_ctx* ctx, double* out);

/* Advance one step and copy its intermediates (each may be NULL), all
 * [18][n_nodes] double: post-collision populations psi_hat (eqn::collide),
 * the lumped-scaled right-hand side b/m of eq:galerkin_lbm, and the solve's
 * increment delta with M11 delta = b (NaN at wall nodes, where the wall
 * operator has already been applied). */
int felbm_step_debug(felbm_ctx* ctx, double* psi_hat, double* rhs_over_m, double* delta);

/* Reduction band for band_ke: nodes with R - w <= |x - (xc, yc)| <= R + w
 * (minimum image in periodic x).  R <= 0 disables it. */
int felbm_set_band(felbm_ctx* ctx, double xc, double yc, double R, double w);

/* FP64 reductions of the current state.  Errors: EINVAL, ESTATE. */
int felbm_diagnostics(felbm_ctx* ctx, felbm_diag* out);

/* Sample the residual of the mass-matrix solve every `every` steps (every
 * step whose index is a multiple of `every`); 0 (the default) disables it.
 * A sampled step ends its solve with a plain sweep, an FP64 residual
 * reduction and a separate update; its populations are bitwise those of an
 * unsampled step.  Errors: EINVAL (every < 0). */
int felbm_set_residual_sampling(felbm_ctx* ctx, int64_t every);

/* felbm_diagnostics for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same reductions, bitwise the same results, with the block
 * partials, the reduced record and the non-finite flag in a fixed scratch
 * array of 1.5 MiB per device, held until the process ends, instead of
 * memory allocated per call.  Calls no allocating routine.  Every call on a
 * device shares that device's scratch, so calls that overlap on one device
 * (several host threads, or streams not ordered against each other) race.
 * The last call's contents stay in the scratch.
 * Errors: EINVAL (null output, more than 8,388,608 nodes, or the
 * collision-step nodal force scheme), ESTATE, EDEVICE. */
int felbm_diagnostics_noalloc(felbm_ctx* ctx, felbm_diag* out);

/* Per-step history of the FP64 reductions computed inside the step (mass,
 * mean KE, max |u| of the state entering each step), most recent last.
 * Copies min(max_entries, available) records; *n_out receives the count. */
int felbm_history(felbm_ctx* ctx, felbm_diag* out, int64_t max_entries, int64_t* n_out);

/* Checkpoint of the state: felbm_state_bytes gives the buffer size; save
 * copies the populations (compute precision, internal layout) and the step
 * counter to buf; load restores them.  Errors: EINVAL (null or short
 * buffer, header mismatch), ESTATE. */
int64_t felbm_state_bytes(const felbm_ctx* ctx);
int felbm_save_state(felbm_ctx* ctx, void* buf, int64_t bytes);
int felbm_load_state(felbm_ctx* ctx, const void* buf, int64_t bytes);

/* Run all subsequent device work on this HIP stream (hipStream_t, NULL =
 * the library's own stream).  The stream is not owned by the library. */
int felbm_bind_stream(felbm_ctx* ctx, void* hip_stream);

/* ---- adjoint (reverse mode) ------------------------------------------------
 * Gradients of a loss of the final composition with respect to the per-node
 * wetting potential Omega_c (the parameter of eq. bc2 and Young's relation,
 * Sec. II.B), by a hand-written vector-Jacobian product of every step.
 *
 * felbm_forward_ckpt: advance n_steps >= 1 from the current state (like
 *   felbm_step) and keep the state every `every` steps on the device
 *   (ceil(n_steps/every) + every states of 18 populations per node).
 * felbm_backward: reverse the last felbm_forward_ckpt run.  dL_dC_dev
 *   [n_nodes] (device, caller node order, double) is dL/dC of the final
 *   composition C = sum_a h_a; dL_domega_dev [n_nodes] (device, caller order,
 *   double) receives dL/dOmega_c (nonzero at wall nodes only).  Segments
 *   between checkpoints are recomputed forward; the final state and the step
 *   counter are restored afterwards.  Runs on the bound stream and waits.
 *   Errors: ESTATE (no forward_ckpt run), EINVAL, EDEVICE.
 * felbm_backward_host: the same with host arrays. */
int felbm_forward_ckpt(felbm_ctx* ctx, int64_t n_steps, int64_t every);
int felbm_backward(felbm_ctx* ctx, const double* dL_dC_dev, double* dL_domega_dev);

/* Identifier (> 0) of the felbm_forward_ckpt run that felbm_backward would
 * reverse, or 0 if there is none: every call that changes the state or the
 * wetting field (felbm_set_wetting, felbm_init, felbm_step, felbm_step_async,
 * felbm_step_debug, felbm_load_state, a failed felbm_forward_ckpt) discards
 * the checkpoints, after which felbm_backward returns ESTATE.  A caller that
 * keeps a run for later (an autograd graph) stores the identifier and checks
 * it before reversing.  felbm_backward itself restores the run's final state
 * on every exit path, including errors.  Errors: EINVAL (null). */
int felbm_adjoint_run(const felbm_ctx* ctx, int64_t* run_id);
int felbm_backward_host(felbm_ctx* ctx, const double* dL_dC, double* dL_domega);

/* The same with a general seed (host arrays, caller order): dL/dpsi_bar of
 * the final populations dL_dpsi [18][n_nodes] (may be NULL) plus dL_dC
 * [n_nodes] (may be NULL) added to every h_a; outputs dL_domega [n_nodes] and,
 * if not NULL, dL/dpsi_bar of the populations the run started from,
 * dL_dpsi0 [18][n_nodes]. */
int felbm_backward_full(felbm_ctx* ctx, const double* dL_dpsi, const double* dL_dC, double* dL_domega,
                        double* dL_dpsi0);

/* Lumped mass vector m_i = int phi_i (row sums of M11) in caller order, for
 * losses such as int C dx = sum_i m_i C_i.  Errors: EINVAL, ESTATE. */
int felbm_lumped_mass(felbm_ctx* ctx, double* out);

/* Per-kernel timing with HIP events recorded around every launch of the
 * step's kernels (for measurement; adds event records to the stream). */
typedef struct {
  char name[32];
  int64_t launches;
  double total_ms;
  double bytes_per_launch;   /* algorithmic bytes moved by one launch */
} felbm_kstat;
int felbm_kernel_timing(felbm_ctx* ctx, int32_t enable);
int felbm_kernel_stats(felbm_ctx* ctx, felbm_kstat* out, int32_t max_entries, int32_t* n_out);

/* Sizes of the uploaded mesh and of the consistent mass matrix. */
int felbm_mesh_info(const felbm_ctx* ctx, int64_t* n_nodes, int64_t* n_tris, int64_t* n_wall_edges,
                    int64_t* mass_matrix_offdiag_nnz);

/* Validate a mesh with the same host checks as felbm_upload_mesh, without a
 * context or a device.  msg (may be NULL) receives a message of at most
 * msg_len bytes including the terminator.  Returns FELBM_OK, EINVAL or EMESH. */
int felbm_validate_mesh(int64_t n_nodes, const double* xy, int64_t n_tris, const int32_t* tri,
                        int64_t n_wall_edges, const int32_t* wall_edge, double period_x, char* msg,
                        int32_t msg_len);

void felbm_destroy(felbm_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* FELBM_H */
