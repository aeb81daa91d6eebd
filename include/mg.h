/*
 * mg.h — C ABI of the MI355X (gfx950) geometric-multigrid engine for the
 * elliptic solves of fluid streamer simulation (Marskar, "Adaptive
 * multiscale methods for 3D streamer discharges in air").
 *
 * Every context solves one cell-centred elliptic equation
 *
 *     a u - div(beta grad u) = f        on nx*ny*nz cubic cells of side h,
 *
 * which covers both elliptic families of the paper's model (Sec. 2):
 *   - the potential: the Poisson equation of the model, in the
 *     variable-permittivity form -div(eps grad phi) = rho (a = 0,
 *     beta = eps, f = rho with eps0 = 1);
 *   - each photon group of the three-term radiative-transfer model in its
 *     diffusive (Eddington) form: multiplying that equation by 3 kappa_j
 *     gives (kappa^2 - lap) Psi = f with kappa = sqrt(3) kappa_j and
 *     f = 3 kappa_j eta_j / c (a = kappa^2, beta = 1).
 *
 * Discretisation: second-order cell-centred finite volumes (Sec. 2,
 * spatial discretisation items (ii)-(iii)): interior faces use the harmonic
 * mean 2 beta_P beta_N / (beta_P + beta_N); a Dirichlet face with value g
 * uses the linear ghost 2g - u_P with the boundary cell's beta; a Neumann
 * face has zero flux (the live/grounded electrode faces and zero-flux side
 * walls of Secs. 3-4 are Dirichlet/Neumann faces).
 *
 * Solver: geometric multigrid V-cycles with red-black Gauss-Seidel smoothing
 * (Sec. 2, item (ii)), matrix-free, all steps in hand-written HIP kernels.
 * Coarse operators are rediscretised (coarse face coefficient = mean of the
 * four fine faces it covers), restriction averages the 8 children,
 * prolongation is cell-centred trilinear.  Levels whose largest dimension
 * is at most `bottom_max` are solved by one LDS-resident workgroup in FP64,
 * which continues the V-cycle down to the coarsest grid and solves that
 * grid exactly by conjugate gradients (A is symmetric positive definite).
 *
 * Array layout (every field): C order [nz][ny][nx], x fastest, contiguous,
 * FP64, resident in device memory (hipMalloc'ed or from torch).  The
 * library never keeps a caller pointer beyond the call that receives it.
 *
 * Return codes: MG_OK (0), MG_NOT_CONVERGED (1: soft, x holds the last
 * iterate and the stats are valid), negative values are hard errors whose
 * text is available from mg_last_error() on the calling thread.
 *   MG_EINVAL    invalid argument; x is left untouched
 *   MG_ENOMEM    device allocation failed
 *   MG_EDEVICE   a HIP runtime call failed
 *   MG_EDIVERGED non-finite or growing residual; x is unspecified
 *
 * Threading: one context must not be used from two threads at once;
 * distinct contexts are independent.  All device work of a context is
 * enqueued on the stream given to mg_create; mg_solve and
 * mg_solve_batched return after that work has completed (they report
 * convergence).
 */
#ifndef MG_H_INCLUDED
#define MG_H_INCLUDED

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mg_ctx mg_ctx; /* opaque, owned by the library */

enum {
    MG_OK = 0,
    MG_NOT_CONVERGED = 1,
    MG_EINVAL = -1,
    MG_ENOMEM = -2,
    MG_EDEVICE = -3,
    MG_EDIVERGED = -4
};

enum { MG_BC_DIRICHLET = 0, MG_BC_NEUMANN = 1 };

/* Arithmetic of the solve.
 *   MG_FP64     FP64 V-cycles.
 *   MG_FP32_IR  FP64 iterative refinement: FP64 residual, correction update
 *               and bottom solve; the inner V-cycle smooths and transfers
 *               in FP32.
 *   MG_BF16_IR  as MG_FP32_IR with BF16 storage of the inner fields
 *               (coefficients FP32; FP32 arithmetic, round-to-nearest-even).
 * Every precision converges to the same FP64 solution. */
enum { MG_FP64 = 0, MG_FP32_IR = 1, MG_BF16_IR = 2 };

/* mg_solve flags */
enum {
    MG_GUESS = 1u /* x holds an initial guess.  It is kept only if, after
                     the nu1 pre-smoothing sweeps that open every cycle
                     (FP64, finest level), its residual does not exceed
                     that of the zero guess: ||b - A S(x)|| <= ||b||.
                     Otherwise the solve starts from zero and
                     stats.fell_back = 1.  (Grids handled by the bottom
                     solver alone, or nu1 = 0: the raw residual
                     ||b - A x|| is compared.)  stats.rel_res0 is the
                     relative residual of the guess at that test (1
                     after a fallback). */
};

typedef struct {
    int nx, ny, nz;  /* cells per axis, >= 1 each; nx*ny <= 2^28 and
                        nx*ny*nz <= 4e9 */
    double h;        /* cell side, > 0 */
    int precision;   /* MG_FP64 | MG_FP32_IR | MG_BF16_IR */
    int nu1, nu2;    /* red-black Gauss-Seidel sweeps before/after the
                        coarse correction, 0..8 each, nu1 + nu2 >= 1 */
    int bottom_max;  /* levels with max dimension <= bottom_max go to the
                        single-workgroup bottom solver; 2..16 */
    int max_cycles;  /* V-cycles (outer refinement steps) per solve, >= 1 */
    double rtol;     /* stop when ||b - A x||_2 <= rtol ||b||_2 */
} mg_desc;

/* Face order everywhere: x-, x+, y-, y+, z-, z+. */
typedef struct {
    int type[6];     /* MG_BC_DIRICHLET | MG_BC_NEUMANN */
    double value[6]; /* Dirichlet value g (ignored for Neumann) */
} mg_bcs;

typedef struct {
    int cycles;        /* V-cycles (or refinement steps) performed */
    double rel_res0;   /* ||b - A x0|| / ||b|| of the starting iterate
                          (1 for a zero start; for MG_GUESS see there) */
    double rel_res;    /* final ||b - A x|| / ||b|| (FP64) */
    int fell_back;     /* 1 if an MG_GUESS was rejected */
    double ms;         /* wall time of the call */
} mg_stats;

/* Fill d with the defaults for an nx*ny*nz grid of side h: MG_FP64,
 * V(2,2), bottom_max 16, max_cycles 50, rtol 1e-10. */
void mg_desc_default(mg_desc *d, int nx, int ny, int nz, double h);

/* Create a context: validates d, builds the level hierarchy (every axis is
 * halved while all axes are even and the largest exceeds 1) and allocates
 * the device buffers.  The grid must reach a level whose largest dimension
 * is <= d->bottom_max with at most 4096 cells, otherwise MG_EINVAL.
 * hip_stream: a hipStream_t (NULL = the default stream).  *out receives
 * the context; it is NULL on error. */
int mg_create(const mg_desc *d, void *hip_stream, mg_ctx **out);

/* Set the operator: eps_dev = device array of nx*ny*nz cell coefficients
 * (beta; NULL means beta = 1), copied into library storage; a >= 0 the
 * screening coefficient kappa^2; bc the six face conditions.  Errors
 * (MG_EINVAL): eps outside (0, 1e100] (checked on the device), a < 0
 * or not finite, an unknown face type, or a singular operator (a == 0 and
 * no Dirichlet face). */
int mg_set_coeffs(mg_ctx *c, const double *eps_dev, double a, const mg_bcs *bc);

/* Solve A x = b with b = f + boundary terms.  f_dev and x_dev are device
 * arrays of nx*ny*nz FP64 values; f_dev is read only; x_dev receives the
 * solution (without MG_GUESS its input content is ignored).  st may be
 * NULL.  A non-finite f is MG_EINVAL; a non-finite guess is rejected like
 * any other guess worse than zero (MG_EINVAL where the raw residual is
 * compared). */
int mg_solve(mg_ctx *c, const double *f_dev, double *x_dev, unsigned flags, mg_stats *st);

/* Solve `count` independent problems (contexts may differ in size and
 * coefficients; all must share one stream and one precision).  The
 * V-cycle levels of all problems advance together: each level phase of
 * the whole batch is one kernel launch over a work list of tiles, the
 * cycle is captured once into a hipGraph and replayed, and converged
 * problems are skipped on the device.  f_dev[i], x_dev[i] as in mg_solve
 * for context c[i]; st (optional) receives count entries.  With MG_GUESS
 * each guess is screened on its raw residual (||b - A x|| <= ||b||). */
int mg_solve_batched(int count, mg_ctx *const *c, const double *const *f_dev,
                     double *const *x_dev, unsigned flags, mg_stats *st);

/* Free a context and all its device memory (NULL is accepted). */
int mg_destroy(mg_ctx *c);

/* Text of the last hard error raised on the calling thread ("" if none). */
const char *mg_last_error(void);

/* ------------------------------------------------------------------ *
 * Building blocks exposed for verification and for callers that drive
 * their own iterations.  Same arrays and rules as mg_solve.
 * ------------------------------------------------------------------ */

/* r_dev = b - A x (b = f + boundary terms, FP64); *rnorm = ||r||_2 and
 * *bnorm = ||b||_2 (either may be NULL).  r_dev may be NULL (norms only). */
int mg_residual(mg_ctx *c, const double *f_dev, const double *x_dev, double *r_dev,
                double *rnorm, double *bnorm);

/* Apply `sweeps` red-black Gauss-Seidel sweeps (red = (i+j+k) even first,
 * then black) of the finest-level equation to x_dev in place, FP64. */
int mg_smooth(mg_ctx *c, const double *f_dev, double *x_dev, int sweeps);

/* u_dev (level l) += P e_dev (level l+1): the cell-centred trilinear
 * prolongation of a coarse correction, ghost values reflected across the
 * box faces and negated at Dirichlet faces (paper Sec. 2, the V-cycle's
 * interpolation step), FP64.  Dimensions from mg_level_dims; requires
 * 0 <= l < mg_num_levels - 1. */
int mg_prolong_add(mg_ctx *c, int l, const double *e_dev, double *u_dev);

/* Number of levels and the dimensions of level l (0 = finest). */
int mg_num_levels(const mg_ctx *c);
int mg_level_dims(const mg_ctx *c, int l, int *nx, int *ny, int *nz);

/* Kernel tile selection for the finest-level smoother: tile = 0 picks the
 * built-in heuristic, 1..MG_NUM_TILES selects a fixed (TX, TY) variant;
 * zchunk = planes per workgroup (0 = heuristic).  Used by the autotuner. */
#define MG_NUM_TILES 6
int mg_set_tiling(mg_ctx *c, int tile, int zchunk);
/* (TX, TY) of tile variant t (1..MG_NUM_TILES). */
int mg_tile_shape(int t, int *tx, int *ty);

/* Autotune: time every tile variant and z-chunk of the finest-level
 * smoother for this context's grid, precision and coefficients (one sweep
 * each, `reps` repetitions on the context's stream) and keep the fastest.
 * Writes the chosen variant to *tile, *zchunk and its time per sweep in
 * microseconds to *us (any may be NULL).  Requires mg_set_coeffs. */
int mg_autotune(mg_ctx *c, int reps, int *tile, int *zchunk, double *us);

/* Measurement hook: while enabled, every launch of the finest-level
 * smoother is bracketed by HIP events on the context's stream and, after
 * each solve, its duration and algorithmic bytes (cells x bytes read and
 * written once) are accumulated.  Enabling resets the counters. */
int mg_timing(mg_ctx *c, int enable);
/* Accumulated launches, total milliseconds and total algorithmic bytes;
 * *kernel (may be NULL) receives a static description of the kernel. */
int mg_timing_read(const mg_ctx *c, long *launches, double *ms, double *bytes, const char **kernel);

#ifdef __cplusplus
}
#endif
#endif /* MG_H_INCLUDED */
