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
 *   MG_EDIVERGED the residual diverged: it is not finite, or it exceeds
 *                1e6 times the starting one, or it grew in each of 4
 *                consecutive cycles to more than 10 times the smallest
 *                residual of the solve; x is unspecified and the stats hold
 *                the cycle and residual at which this was seen.  (A solve
 *                that stalls at its rounding floor moves by small factors
 *                and ends with MG_NOT_CONVERGED instead.)
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

/* Create a context for one cell-centred elliptic equation on an
 * nx x ny x nz grid (paper Sec. 2, spatial-discretisation items (ii)-(iii):
 * the Poisson and radiative-transfer equations on Cartesian cells, solved by
 * geometric multigrid): validates d, builds the level hierarchy (every axis is
 * halved while all axes are even and the largest exceeds 1) and allocates
 * the device buffers.  The grid must reach a level whose largest dimension
 * is <= d->bottom_max with at most 4096 cells, otherwise MG_EINVAL.
 * hip_stream: a hipStream_t (NULL = the default stream).  *out receives
 * the context; it is NULL on error. */
int mg_create(const mg_desc *d, void *hip_stream, mg_ctx **out);

/* Set the operator a u - div(beta grad u) of Sec. 2's model equations: the
 * potential (Eq. (streamer_equations), second line, with the permittivity as
 * beta, a = 0) or a photon group of the three-term radiative-transfer model
 * (Eq. (rte) times 3 kappa_j: beta = 1, a = kappa^2); bc gives the electrode (Dirichlet) and
 * zero-flux (Neumann) faces of the set-ups of Secs. 3-4.
 * eps_dev = device array of nx*ny*nz cell coefficients (beta; NULL means
 * beta = 1), copied into library storage; a >= 0 the screening coefficient
 * kappa^2; bc the six face conditions.  Errors (MG_EINVAL): eps outside
 * (0, 1e100] (checked on the device), a < 0 or not finite, an unknown face
 * type, or a singular operator (a == 0 and no Dirichlet face).
 * MG_FP32_IR and MG_BF16_IR contexts run their inner cycle on the
 * coefficients times a power of two that centres them on 1; they reject
 * (MG_EINVAL) coefficients whose largest and smallest value differ by more
 * than 2^70 (about 1.2e21), and a above 2^100 times that scale: use MG_FP64
 * for such operators. */
int mg_set_coeffs(mg_ctx *c, const double *eps_dev, double a, const mg_bcs *bc);

/* Set an operator whose face coefficients are given directly: the
 * face-centred diffusion coefficient D of the implicit diffusion solves
 * (Sec. 2, item (ii): cell-centred discretisation of div(D grad n) with the
 * coefficient on the faces).  bx_dev, by_dev, bz_dev are device arrays of
 * (nx+1)*ny*nz, nx*(ny+1)*nz and nx*ny*(nz+1) FP64 values, laid out as
 *     bx[(k*ny + j)*(nx+1) + i]   the face between cells i-1 and i, i = 0..nx
 *     by[(k*(ny+1) + j)*nx + i]   j = 0..ny
 *     bz[(k*ny + j)*nx + i]       k = 0..nz (nz+1 planes)
 * and copied into library storage; the entries on the box faces are the
 * coefficients of Dirichlet terms (unused on Neumann faces).  a, bc and the
 * errors as mg_set_coeffs; every entry must lie in (0, 1e100] (checked on
 * the device).  MG_FP64 contexts only (MG_EINVAL otherwise).  Coarser levels
 * average the four fine faces each coarse face covers. */
int mg_set_face_coeffs(mg_ctx *c, const double *bx_dev, const double *by_dev, const double *bz_dev, double a,
                       const mg_bcs *bc);

/* Stored face coefficients plus a per-cell extra diagonal d: the operator
 * (a + d_P) u - div(beta grad u), as mg_set_face_coeffs with d (device,
 * nx*ny*nz FP64 in [0, 1e100], copied) and faces allowed to vanish (in
 * [0, 1e100]); coarse levels take the mean of the 8 children's d.  This is
 * the symmetric part of a cut-cell operator (Sec. 2, the embedded boundary
 * formalism): faces scaled by their gas apertures, the embedded face's
 * diagonal and identity rows for covered cells, used to precondition the
 * cut-cell solves of mge.h.  MG_FP64 contexts only; every cell needs
 * a + d + h^-2 (its interior and Dirichlet faces) > 0, else MG_EINVAL.
 * mg_solve_batched rejects such contexts. */
int mg_set_face_coeffs_diag(mg_ctx *c, const double *bx_dev, const double *by_dev, const double *bz_dev,
                            const double *d_dev, double a, const mg_bcs *bc);

/* Solve A x = b with b = f + boundary terms by V-cycles (Sec. 2, item (ii):
 * geometric multigrid with red-black Gauss-Seidel smoothing and a Krylov
 * bottom solver) until ||b - A x||_2 <= rtol ||b||_2.  f_dev and x_dev are
 * device arrays of nx*ny*nz FP64 values; f_dev is read only; x_dev receives the
 * solution (without MG_GUESS its input content is ignored).  st may be
 * NULL.  A non-finite f is MG_EINVAL; a non-finite guess is rejected like
 * any other guess worse than zero (MG_EINVAL where the raw residual is
 * compared). */
int mg_solve(mg_ctx *c, const double *f_dev, double *x_dev, unsigned flags, mg_stats *st);

/* Solve `count` independent problems of the kind mg_solve solves (for
 * instance the four elliptic solves of one field update of Sec. 2.1, or
 * many grid patches); contexts may differ in size and coefficients; all must
 * share one stream and one precision.  The
 * V-cycle levels of all problems advance together: each level phase of
 * the whole batch is one kernel launch over a work list of tiles, the
 * cycle is captured once into a hipGraph and replayed, and converged
 * problems are skipped on the device.  f_dev[i], x_dev[i] as in mg_solve
 * for context c[i]; st (optional) receives count entries.  With MG_GUESS
 * each guess is screened on its raw residual (||b - A x|| <= ||b||).
 * Returns MG_EDIVERGED if any problem diverged (that problem is stopped, the
 * others run on; st[i] tells which), else MG_NOT_CONVERGED if any problem
 * did not converge, else MG_OK. */
int mg_solve_batched(int count, mg_ctx *const *c, const double *const *f_dev,
                     double *const *x_dev, unsigned flags, mg_stats *st);

/* One implicit diffusion advance of the paper's TGA scheme (Sec. 2.1,
 * step (vi), Eq. (tga)):
 *     (I - mu1 L)(I - mu2 L) out = (I + mu3 L) n,   L u = div(beta grad u),
 * with beta the context's coefficients (face D from mg_set_face_coeffs, or a
 * cell coefficient, or 1) and zero flux on every face (the context's bc must
 * be all Neumann, else MG_EINVAL).  The coefficients are those of Twizell,
 * Gumel and Arigu: q = 2 - sqrt(2) - 1e-6, r = sqrt(q^2 - 4q + 2),
 * mu1 = (q - r)/2 dt, mu2 = (q + r)/2 dt, mu3 = (1 - q) dt (second order, and
 * the amplification vanishes for stiff modes).  Two Helmholtz solves, each
 * as mg_solve with the context's precision, rtol and max_cycles: first
 * (1/mu1) y - div(beta grad y) = (I + mu3 L) n / mu1, then
 * (1/mu2) out - div(beta grad out) = y / mu2.  The context's a is used as
 * 1/mu1 and 1/mu2 during the call and restored afterwards.  n_dev, out_dev:
 * distinct device arrays of nx*ny*nz FP64 values (n read only).  flags:
 * MG_GUESS starts the first solve from n and the second from y (each
 * screened as in mg_solve), else both start from zero.  st (optional)
 * receives two entries, one per solve.  Returns the worse of the two
 * solves' codes. */
int mg_tga_step(mg_ctx *c, double dt, const double *n_dev, double *out_dev, unsigned flags, mg_stats *st);

/* Free a context and all its device memory (NULL is accepted).  Returns
 * MG_OK. */
int mg_destroy(mg_ctx *c);

/* Text of the last hard error raised on the calling thread ("" if none).
 * The message is kept per thread, not per context, so that it also reports
 * errors of calls that have no context yet (mg_create) or several
 * (mg_solve_batched); the pointer stays valid until the thread's next
 * failing call. */
const char *mg_last_error(void);

/* ------------------------------------------------------------------ *
 * Building blocks exposed for verification and for callers that drive
 * their own iterations.  Same arrays and rules as mg_solve.
 * ------------------------------------------------------------------ */

/* r_dev = b - A x (b = f + boundary terms, FP64); *rnorm = ||r||_2 and
 * *bnorm = ||b||_2 (either may be NULL).  r_dev may be NULL (norms only). */
int mg_residual(mg_ctx *c, const double *f_dev, const double *x_dev, double *r_dev,
                double *rnorm, double *bnorm);

/* y_dev = alpha x_dev + beta A x_dev, with A the finest-level operator and
 * zero boundary values (the matrix of the discretisation, Sec. 2 items
 * (ii)-(iii)); x and y distinct FP64 device arrays of nx*ny*nz values. */
int mg_apply(mg_ctx *c, double alpha, double beta, const double *x_dev, double *y_dev);

/* The electric field and the dielectric relaxation time of the multirate
 * scheme (Sec. 2.2; the time-step table's dt_E = eps0 |E| / |J|): with the
 * potential phi_dev of this context's grid and boundary conditions (the
 * solution of an mg_solve of the potential),
 *     E = -grad(phi)  at the cell centres, by central differences over two
 *                     cells, with the discretisation's ghost values beyond
 *                     the box (2g - phi beyond a Dirichlet face of value g,
 *                     phi beyond a Neumann face),
 *     J = sigma E     the drift current of the cell conductivity sigma_dev
 *                     (sigma = e mu_e n_e for electrons; NULL: no current),
 *     *emax = max |E|, *jmax = max |J| over the grid,
 *     *dt_e = eps0 * max|E| / max|J| (infinity where there is no current),
 * the largest values over the grid giving one step size for the domain.
 * ex_dev, ey_dev, ez_dev (nx*ny*nz FP64 each, any may be NULL) receive the
 * components of E; emax, jmax, dt_e are host pointers (any may be NULL).
 * eps0 > 0 in the units of the potential equation (1 where eps0 is folded
 * into the source, as in mg_set_coeffs). */
int mg_field(mg_ctx *c, const double *phi_dev, const double *sigma_dev, double eps0, double *ex_dev,
             double *ey_dev, double *ez_dev, double *emax, double *jmax, double *dt_e);

/* The multirate schedule of Sec. 2.2: the elliptic equations are re-solved
 * once per coarse step dt_c = m dt_fine with m the largest integer such that
 * dt_c <= alpha dt_e (at least 1): the advective-reactive part takes m fine
 * steps between two field updates.  *m receives m (capped at 1e9). */
int mg_relaxation_substeps(double dt_fine, double dt_e, double alpha, int *m);

/* Apply `sweeps` red-black Gauss-Seidel sweeps (red = (i+j+k) even first,
 * then black) of the finest-level equation to x_dev in place, FP64. */
int mg_smooth(mg_ctx *c, const double *f_dev, double *x_dev, int sweeps);

/* Storage types of mg_smooth_level. */
enum { MG_STORE_F64 = 0, MG_STORE_F32 = 1, MG_STORE_BF16 = 2 };

/* `sweeps` fused red-black Gauss-Seidel sweeps (Sec. 2, item (ii); red =
 * (i+j+k) even first) of the equation of level l, in the storage type a
 * solve uses there: level 0 in MG_STORE_F64 is the finest equation with its
 * boundary values (as mg_smooth); every other (level, storage) pair is the
 * homogeneous correction equation that the V-cycle smooths, with the level's
 * coefficients (level 0: the cell coefficient; coarser levels: the averaged
 * face coefficients).  MG_STORE_F32 / MG_STORE_BF16 need an MG_FP32_IR /
 * MG_BF16_IR context and use its FP32 coefficient copies (levels below the
 * bottom-solver level only, for cell coefficients).  b_dev and x_dev are FP64
 * device arrays with the dimensions of level l (mg_level_dims): both are
 * rounded to the storage type (to nearest even), swept on library buffers,
 * and x is converted back to FP64.  tile (0 = heuristic, 1..MG_NUM_TILES) and
 * zchunk (planes per workgroup, 0 = heuristic) select the launch.  For
 * verification; it synchronises the context's stream. */
int mg_smooth_level(mg_ctx *c, int l, int store, const double *b_dev, double *x_dev, int sweeps, int tile,
                    int zchunk);

/* Options of mg_set_option. */
enum {
    MG_OPT_CORRECTION_WEIGHT = 1 /* the coarse-grid correction is added to
                                    the finest level as u += w * P e;
                                    w in (0, 4], default 1 (the plain
                                    V-cycle).  w > 2 over-corrects the
                                    smooth error components, which then
                                    grow: used to exercise the divergence
                                    test. */
};
int mg_set_option(mg_ctx *c, int key, double value);

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

/* ------------------------------------------------------------------ *
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * ------------------------------------------------------------------ */

/* Bytes of the library's file-scope device array that holds the partial
 * sums of mg_residual_noalloc's reductions (one copy per GPU, kept until the
 * process ends): 2048 workgroup pairs plus 8 result slots. */
#define MG_NOALLOC_SCRATCH_BYTES 32832

/* mg_residual without a context and without allocating: r_dev = b - A x and
 * the norms ||b - A x||_2, ||b||_2 (b = f + boundary terms), for the grid of
 * d (only nx, ny, nz and h are read), the cell coefficient eps_dev (NULL = 1;
 * its entries must lie in (0, 1e100], checked on the device), a and bc as in
 * mg_set_coeffs.  f_dev, x_dev, r_dev as in mg_residual (r_dev may be NULL);
 * rnorm, bnorm host pointers (either may be NULL).  hip_stream: the stream
 * (NULL = default) whose device is the current device.  Calls no hipMalloc
 * or hipFree and keeps no pointer.  Grid limits and errors as in mg_create
 * and mg_set_coeffs; the scratch of MG_NOALLOC_SCRATCH_BYTES serves every
 * grid size (each reduction uses at most 2048 workgroups).  All calls on one
 * GPU share its scratch array: calls that overlap in time on the same GPU
 * (two host threads, or two streams) race and must be serialised by the
 * caller.  It synchronises the stream before it returns. */
int mg_residual_noalloc(const mg_desc *d, const double *eps_dev, double a, const mg_bcs *bc,
                        const double *f_dev, const double *x_dev, double *r_dev, double *rnorm,
                        double *bnorm, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* MG_H_INCLUDED */
