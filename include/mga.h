/*
 * mga.h — composite (two-level AMR) solves of the MI355X multigrid engine.
 *
 * The paper solves its elliptic equations on an adaptive hierarchy of
 * Cartesian patches (Secs. 2-4: a base grid refined by patches of 16^3-32^3
 * cells) with the cell-centred discretisation of Sec. 2, items (ii)-(iii).
 * A context here holds one base grid (an mg_desc, its six box faces) and a
 * set of refinement-ratio-2 patches, and solves the composite problem
 *
 *     a u - div(beta grad u) = f   on the uncovered base cells and on every
 *                                  patch cell,
 *
 * discretised as on one grid inside each level, and across a coarse-fine
 * interface by (1) a ghost value beyond each fine face, G = F/3 + 2/3 C~,
 * where F is the fine cell and C~ the value of the coarse cell holding the
 * ghost moved to the ghost's tangential position by central differences of
 * that cell's tangential coarse neighbours (exact for linear functions), and
 * (2) refluxing: the coarse cell's flux through the face is the sum of the
 * four fine fluxes.  The operator is conservative and not symmetric; it is
 * solved by BiCGStab (the Krylov method the paper names) preconditioned by
 * one multigrid V-cycle of the base grid on the restricted residual plus one
 * V-cycle of each patch with zero correction values on its boundary.
 *
 * Patches ("boxes") are ranges of the level-1 index space (2nx x 2ny x 2nz
 * cells of side h/2): fine cells lo..hi-1 per axis (x, y, z), every bound
 * even (boxes cover whole coarse cells), each box at least one coarse cell
 * inside the domain and at least one coarse cell away from every other box,
 * and each box's dimensions coarsenable like any grid of mg_create.
 *
 * Arrays (all FP64, device, C order [z][y][x]): the base grid as in mg.h;
 * patch p as a (hi-lo) box of its own.  Return codes and mg_last_error as in
 * mg.h.  A context is not thread-safe; it enqueues on the given stream and
 * its calls return after the work has finished.
 */
#ifndef MGA_H_INCLUDED
#define MGA_H_INCLUDED

#include "mg.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mga_ctx mga_ctx; /* opaque, owned by the library */

typedef struct {
    int lo[3]; /* first fine cell per axis (x, y, z), even */
    int hi[3]; /* one past the last fine cell, even */
} mga_box;

/* Create a composite context: base grid d (its rtol and max_cycles are the
 * stopping rule and the iteration cap of mga_solve; precision must be
 * MG_FP64) and nbox >= 0 boxes as above.  Errors: MG_EINVAL for a bad grid
 * or box, MG_ENOMEM. */
int mga_create(const mg_desc *d, int nbox, const mga_box *boxes, void *hip_stream, mga_ctx **out);

/* Set the operator: eps_base (base cells) and eps_fine[p] (cells of box p)
 * the cell coefficients, both given or both NULL (beta = 1), copied into
 * library storage; a and bc as in mg_set_coeffs (bc applies to the base
 * grid's box faces; patches never touch them).  Coefficients must lie in
 * (0, 1e100]. */
int mga_set_coeffs(mga_ctx *m, const double *eps_base, const double *const *eps_fine, double a,
                   const mg_bcs *bc);

/* Solve the composite problem.  f_base and f_fine[p] are the sources (the
 * base values under the boxes are not used); x_base and x_fine[p] receive
 * the solution, the covered base cells the mean of their eight fine
 * children.  flags: MG_GUESS starts from the given x (covered base values
 * ignored), else from zero.  st (optional): cycles = BiCGStab iterations,
 * rel_res0/rel_res = ||b - A u|| / ||b|| at the start and the end (volume-
 * weighted L2 over the unknowns).  MG_NOT_CONVERGED after max_cycles
 * iterations; MG_EDIVERGED on a breakdown or a non-finite residual. */
int mga_solve(mga_ctx *m, const double *f_base, const double *const *f_fine, double *x_base,
              double *const *x_fine, unsigned flags, mg_stats *st);

/* y = A x of the composite operator with zero boundary values (per unit
 * volume; the covered base cells of y are 0, of x ignored).  For
 * verification. */
int mga_apply(mga_ctx *m, const double *x_base, const double *const *x_fine, double *y_base,
              double *const *y_fine);

/* Measurement hook: time the finest-level smoother of the base grid's
 * V-cycles with HIP events on the context's stream (as mg_timing and
 * mg_timing_read of mg.h, for the preconditioner's base-grid context). */
int mga_timing(mga_ctx *m, int enable);
int mga_timing_read(const mga_ctx *m, long *launches, double *ms, double *bytes, const char **kernel);

/* Free a context (NULL accepted). */
int mga_destroy(mga_ctx *m);

#ifdef __cplusplus
}
#endif
#endif /* MGA_H_INCLUDED */
