/*
 * mge.h — embedded-boundary (cut-cell) solves of the MI355X multigrid engine.
 *
 * The paper treats the electrode as an embedded boundary in a Cartesian
 * grid (Sec. 2, the spatial discretisation: finite volumes on cut cells,
 * second-order cell-centred elliptic operators; Sec. 4: a needle electrode
 * protruding from the live top face of the box; Sec. 2.2: curved solid
 * boundaries degrade multigrid convergence).  A context here holds one grid
 * (an mg_desc), its cut-cell geometry and operator, and solves
 *
 *     kappa a u - div(beta grad u) = kappa f   in the gas part of each cell
 *
 * integrated over the cell's gas volume (per unit cell volume):
 *   - face fluxes beta_f alpha_f (u_N - u_P) / h^2, alpha_f the face's gas
 *     fraction (aperture), beta_f the harmonic mean of the cells' beta;
 *   - the box faces as in mg.h (Dirichlet terms weighted by the aperture);
 *   - an embedded face per boundary cell whose area vector closes the
 *     divergence theorem over the cut cell (A n = -sum_f alpha_f n_f h^2),
 *     carrying beta_P A dudn / h^3, where dudn is the derivative along the
 *     normal into the gas at the given surface point x_b (u = g there),
 *     second-order from two points x_b + h nu and x_b + 2 h nu valued by
 *     trilinear interpolation of the cell-centred unknowns;
 *   - covered cells (kappa = 0) hold u = g.
 * The operator is not symmetric.  mge_solve runs BiCGStab (the Krylov
 * method the paper pairs with its multigrid) on it, preconditioned by one
 * V-cycle of the engine on the operator's symmetric part (aperture-weighted
 * faces, the embedded face's diagonal 1.5 beta A / h^2, identity rows on
 * covered cells; mg_set_face_coeffs_diag).  Covered cells start at g and
 * receive no correction.
 *
 * Arrays are FP64 device arrays in C order [z][y][x] unless stated; face
 * arrays use mg_set_face_coeffs's layout (ax [nz][ny][nx+1], ay
 * [nz][ny+1][nx], az [nz+1][ny][nx]).  Return codes and mg_last_error as in
 * mg.h.  A context is not thread-safe; its calls return after their work
 * has finished.
 */
#ifndef MGE_H_INCLUDED
#define MGE_H_INCLUDED

#include "mg.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mge_ctx mge_ctx; /* opaque, owned by the library */

/* Create a context for grid d (precision MG_FP64; rtol and max_cycles are
 * the stopping rule and iteration cap of mge_solve).  Errors: MG_EINVAL,
 * MG_ENOMEM. */
int mge_create(const mg_desc *d, void *hip_stream, mge_ctx **out);

/* Set geometry and operator (all arrays copied into library storage).
 *   kappa  gas volume fraction per cell, in [0, 1];
 *   ax, ay, az  face apertures, in [0, 1];
 *   nb, bidx  the boundary cells: flat C-order cell indices (host array of
 *          nb int64, strictly increasing), each with kappa > 0;
 *   boff   host array [nb][3]: the surface point of each boundary cell
 *          minus its centre, in units of h (x, y, z);
 *   eps    beta per cell in (0, 1e96] (NULL: 1);
 *   a, bc  as in mg_set_coeffs (the box faces);
 *   g      the potential of the embedded surface per cell (device; used on
 *          covered and boundary cells), or NULL for the constant g_eb.
 * Errors: MG_EINVAL for values out of range (message names the array). */
int mge_set_geometry(mge_ctx *e, const double *kappa, const double *ax, const double *ay, const double *az,
                     long nb, const long *bidx, const double *boff, const double *eps, double a,
                     const mg_bcs *bc, const double *g, double g_eb);

/* Solve from zero (or from x with MG_GUESS; covered cells start at g).
 * st: cycles = BiCGStab iterations, rel_res0/rel_res = ||b - A u|| / ||b||
 * over all rows (2-norm).  MG_NOT_CONVERGED after max_cycles iterations,
 * MG_EDIVERGED on a breakdown or a non-finite residual. */
int mge_solve(mge_ctx *e, const double *f, double *x, unsigned flags, mg_stats *st);

/* y = A x (no boundary data: zero box-face values and g = 0); b = the
 * right-hand side of source f (kappa f plus the box-face and embedded
 * terms, g / h^2 on covered cells).  For verification. */
int mge_apply(mge_ctx *e, const double *x, double *y);
int mge_rhs(mge_ctx *e, const double *f, double *b);

/* Measurement hook: the finest-level smoother of the preconditioner's
 * V-cycles, timed with HIP events (as mg_timing / mg_timing_read). */
int mge_timing(mge_ctx *e, int enable);
int mge_timing_read(const mge_ctx *e, long *launches, double *ms, double *bytes, const char **kernel);

/* Free a context (NULL accepted). */
int mge_destroy(mge_ctx *e);

#ifdef __cplusplus
}
#endif
#endif /* MGE_H_INCLUDED */
