/*
 * felbm3d.h — C ABI of the 3-D FE-LBM step on MI355X (gfx950): D3Q19
 * populations g and h (38 per node) on linear tetrahedra, the setting of the
 * paper itself (Matin, Misztal, Hernandez-Garcia, Mathiesen, arXiv:1708.04678,
 * Sec. II.A: D3Q19 lattice; Sec. II.C: linear tetrahedral elements).
 *
 * The step is the one of felbm.h with the tetrahedral forms: moments and BGK
 * collision (eqn::collide); element gradients; the nodal patch Laplacian of
 * C with averaged face gradients and the wetting flux of eq. bc2 integrated
 * exactly over wall faces (eqn:lapl_int_mp); mu (eqn:mp_mu); the element
 * Laplacian of mu (Sec. II.D); P0 forces at barycentric values (eq:G, eq:H,
 * eq:intF) in the Galerkin right-hand side (eq:galerkin_lbm, with
 * b_i = sum_T V_T q_T (dt/4 + dt^2/2 e . grad N_i)); the consistent-mass solve
 * by K Chebyshev-step Richardson sweeps with the lumped-mass preconditioner on
 * the spectrum [1/5, 1] of diag(m)^-1 M11 for P1 tetrahedra; the wall
 * operator (opposite pairs replaced by their mean at wall nodes).
 *
 * Conventions as in felbm.h: int status codes (FELBM_*), host arrays owned by
 * the caller and copied, device memory owned by the library, arrays in the
 * caller's node / tetrahedron order, all validation on the host before any
 * device work, deterministic results (no atomics).  Global-gather kernels on
 * every mesh.  felbm_params is shared with felbm.h: precision FELBM_FP64 or
 * FELBM_FP32 (FP32 populations and arithmetic; FP64 chemical-potential chain,
 * reductions and composition: C = sum_a h_a + r with a per-node FP64
 * remainder r, whose increment is the FP64 zeroth moment of the h right-hand
 * side solved by the same sweeps with exactly mass-preserving column sums, as
 * in felbm.h), solver_sweeps, lambda_min / lambda_max (0/0 selects [1/5, 1]);
 * kernels and force_scheme must be 0.
 */
#ifndef FELBM3D_H
#define FELBM3D_H

#include <stdint.h>

#include "felbm.h"

#ifdef __cplusplus
extern "C" {
#endif

enum { FELBM_FIELD_UZ = 8 };  /* third velocity component (N), 3-D only */

typedef struct felbm3d_ctx felbm3d_ctx;

/* Create a context on the current HIP device.  Errors: EINVAL (as
 * felbm_create, and kernels or force_scheme not 0), EDEVICE, ENOMEM. */
int felbm3d_create(const felbm_params* params, felbm3d_ctx** out);
const char* felbm3d_last_error(const felbm3d_ctx* ctx);

/* Upload a P1 tetrahedral mesh.
 *   xyz        [n_nodes][3] coordinates
 *   tet        [n_tets][4] vertex indices with positive volume after the
 *              unwrap (minimum image of each vertex relative to vertex 0 in
 *              the periodic directions)
 *   wall_face  [n_wall_faces][3] node triples of the solid-wall faces; every
 *              boundary face must be listed, and only those
 *   period_x, period_y  > 0: periodic in that direction with this period
 * Errors: EINVAL, EMESH (index out of range, non-positive volume, a face
 * shared by more than two tetrahedra, an unlisted boundary face, a listed
 * face that is not on the boundary), ESTATE (second call), ENOMEM, EDEVICE. */
int felbm3d_upload_mesh(felbm3d_ctx* ctx, int64_t n_nodes, const double* xyz, int64_t n_tets, const int32_t* tet,
                        int64_t n_wall_faces, const int32_t* wall_face, double period_x, double period_y);

/* Per-node wetting potential Omega_c (cos theta = -Omega_c), read at wall
 * nodes only.  Errors: EINVAL, ESTATE. */
int felbm3d_set_wetting(felbm3d_ctx* ctx, const double* omega_c);

/* Populations at the equilibria of C [N], u [N][3] (NULL = 0), p [N] (NULL =
 * 0), then the wall operator; resets the step counter.  Errors: EINVAL, ESTATE. */
int felbm3d_init(felbm3d_ctx* ctx, const double* C, const double* u, const double* p);

/* Advance n_steps >= 0 steps and wait (ENONFINITE if the per-step check
 * sees a NaN/Inf); the _async form queues the work without waiting. */
int felbm3d_step(felbm3d_ctx* ctx, int64_t n_steps);
int felbm3d_step_async(felbm3d_ctx* ctx, int64_t n_steps);

/* Fields as in felbm_read (C, RHO, P, UX, UY, MU, LAPC per node, LAPMU per
 * tetrahedron) plus FELBM_FIELD_UZ. */
int felbm3d_read(felbm3d_ctx* ctx, int32_t field, double* out);

/* Populations [38][n_nodes] (g_0..g_18, h_0..h_18) as double; the D3Q19
 * order is rest, +x, -x, +y, -y, +z, -z, then the (x,y), (x,z), (y,z) plane
 * diagonals each as (+,+), (-,-), (+,-), (-,+). */
int felbm3d_read_populations(felbm3d_ctx* ctx, double* out);

/* FP64 reductions of the current state: mass = sum_i m_i C_i, mean_ke,
 * max_u (band members 0; solver_sweeps = K, solver_residual = -1). */
int felbm3d_diagnostics(felbm3d_ctx* ctx, felbm_diag* out);

int felbm3d_bind_stream(felbm3d_ctx* ctx, void* hip_stream);

/* Per-kernel timing with HIP events around every launch (felbm_kstat as in
 * felbm.h). */
int felbm3d_kernel_timing(felbm3d_ctx* ctx, int32_t enable);
int felbm3d_kernel_stats(felbm3d_ctx* ctx, felbm_kstat* out, int32_t max_entries, int32_t* n_out);

int felbm3d_mesh_info(const felbm3d_ctx* ctx, int64_t* n_nodes, int64_t* n_tets, int64_t* n_wall_faces,
                      int64_t* mass_matrix_offdiag_nnz);

void felbm3d_destroy(felbm3d_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* FELBM3D_H */
