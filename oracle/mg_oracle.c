/*
 * CPU FP64 oracle for the cell-centred elliptic solves (TEST INFRASTRUCTURE).
 *
 * Only tests/, the smoke check and the benchmark's CPU-baseline leg use this
 * file.  It shares no code with the GPU library and is deliberately plain:
 * sequential loops, no blocking, no fusion.
 *
 * Problem (paper Sec. 2, eqs. for the potential and the radiative transfer;
 * item (iii) of the spatial discretisation: second-order cell-centred finite
 * volumes, same discretisation for Poisson and radiative transfer except for
 * the boundary conditions):
 *
 *     a u - div(beta grad u) = f     on nx*ny*nz cubic cells of side h
 *
 *   - beta: cell coefficient (permittivity), NULL means beta = 1;
 *   - interior face P|N: beta_f = 2 beta_P beta_N / (beta_P + beta_N);
 *   - Dirichlet face with value g: ghost u_g = 2g - u_P, i.e. a flux
 *     2 beta_P (u_P - g) / h (beta of the face = beta of the boundary cell);
 *   - Neumann face: zero flux.
 *
 *   (A u)_P = a u_P + h^-2 [ sum_interior beta_f (u_P - u_N)
 *                            + sum_Dirichlet 2 beta_f u_P ]
 *   b_P     = f_P + h^-2 sum_Dirichlet 2 beta_f g_f
 *
 * The unique solution u* = A^-1 b is reached by two independent routes:
 * conjugate gradients (A is symmetric positive definite) and a geometric
 * multigrid V-cycle with a lexicographic Gauss-Seidel smoother (paper item
 * (ii): geometric multigrid with Gauss-Seidel smoothing).  The coarse
 * operators are rediscretised: a coarse face coefficient is the mean of the
 * four fine faces it covers, `a` is unchanged and the corrections carry
 * homogeneous boundary values.  Restriction averages the 8 children;
 * prolongation is cell-centred trilinear (weights 3/4, 1/4 per axis) with
 * ghost values -e (Dirichlet) or +e (Neumann) beyond the box.
 *
 * Layout: arrays are [nz][ny][nx], x fastest.  Face arrays:
 *   bx[(k*ny + j)*(nx+1) + i], i = 0..nx  (face between cells i-1 and i)
 *   by[(k*(ny+1) + j)*nx + i], j = 0..ny
 *   bz[(k*ny + j)*nx + i],     k = 0..nz  (nz+1 planes)
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_DIRICHLET 0
#define ORC_NEUMANN 1

typedef struct {
    int nx, ny, nz;
    double h, a;
    double *bx, *by, *bz; /* face coefficients, owned */
    int bc_type[6];       /* x-, x+, y-, y+, z-, z+ */
} orc_level;

static size_t ncell(const orc_level *L) { return (size_t)L->nx * L->ny * L->nz; }
static size_t idx(const orc_level *L, int i, int j, int k) {
    return ((size_t)k * L->ny + j) * L->nx + i;
}
static double *bxp(const orc_level *L, int i, int j, int k) {
    return &L->bx[((size_t)k * L->ny + j) * (L->nx + 1) + i];
}
static double *byp(const orc_level *L, int i, int j, int k) {
    return &L->by[((size_t)k * (L->ny + 1) + j) * L->nx + i];
}
static double *bzp(const orc_level *L, int i, int j, int k) {
    return &L->bz[((size_t)k * L->ny + j) * L->nx + i];
}

static void level_alloc(orc_level *L) {
    L->bx = (double *)calloc((size_t)(L->nx + 1) * L->ny * L->nz, sizeof(double));
    L->by = (double *)calloc((size_t)L->nx * (L->ny + 1) * L->nz, sizeof(double));
    L->bz = (double *)calloc((size_t)L->nx * L->ny * (L->nz + 1), sizeof(double));
}
static void level_free(orc_level *L) {
    free(L->bx);
    free(L->by);
    free(L->bz);
}

static double harm(double p, double q) { return 2.0 * p * q / (p + q); }

/* Coefficients of the finest level: a cell coefficient eps (NULL = 1) whose
 * faces are formed below, or face coefficients given directly (bx != NULL,
 * layout as in the header comment; boundary entries are the coefficients
 * of the Dirichlet terms), as the diffusion solves of the paper's implicit
 * (TGA) step use them: a face-centred D. */
typedef struct {
    const double *eps;
    const double *bx, *by, *bz;
} orc_coef;

static orc_coef cell_coef(const double *eps) {
    orc_coef c = {eps, NULL, NULL, NULL};
    return c;
}
static orc_coef face_coef(const double *bx, const double *by, const double *bz) {
    orc_coef c = {NULL, bx, by, bz};
    return c;
}

/* Finest-level face coefficients from the cell coefficient. */
static void level0_faces(orc_level *L, const double *eps) {
    for (int k = 0; k < L->nz; ++k)
        for (int j = 0; j < L->ny; ++j)
            for (int i = 0; i <= L->nx; ++i) {
                double v;
                if (!eps) v = 1.0;
                else if (i == 0) v = eps[idx(L, 0, j, k)];
                else if (i == L->nx) v = eps[idx(L, L->nx - 1, j, k)];
                else v = harm(eps[idx(L, i - 1, j, k)], eps[idx(L, i, j, k)]);
                *bxp(L, i, j, k) = v;
            }
    for (int k = 0; k < L->nz; ++k)
        for (int j = 0; j <= L->ny; ++j)
            for (int i = 0; i < L->nx; ++i) {
                double v;
                if (!eps) v = 1.0;
                else if (j == 0) v = eps[idx(L, i, 0, k)];
                else if (j == L->ny) v = eps[idx(L, i, L->ny - 1, k)];
                else v = harm(eps[idx(L, i, j - 1, k)], eps[idx(L, i, j, k)]);
                *byp(L, i, j, k) = v;
            }
    for (int k = 0; k <= L->nz; ++k)
        for (int j = 0; j < L->ny; ++j)
            for (int i = 0; i < L->nx; ++i) {
                double v;
                if (!eps) v = 1.0;
                else if (k == 0) v = eps[idx(L, i, j, 0)];
                else if (k == L->nz) v = eps[idx(L, i, j, L->nz - 1)];
                else v = harm(eps[idx(L, i, j, k - 1)], eps[idx(L, i, j, k)]);
                *bzp(L, i, j, k) = v;
            }
}

/* Coarse face coefficient = mean of the 4 fine faces it covers. */
static void coarsen_faces(const orc_level *F, orc_level *C) {
    for (int k = 0; k < C->nz; ++k)
        for (int j = 0; j < C->ny; ++j)
            for (int i = 0; i <= C->nx; ++i) {
                double s = 0.0;
                for (int dk = 0; dk < 2; ++dk)
                    for (int dj = 0; dj < 2; ++dj) s += *bxp(F, 2 * i, 2 * j + dj, 2 * k + dk);
                *bxp(C, i, j, k) = 0.25 * s;
            }
    for (int k = 0; k < C->nz; ++k)
        for (int j = 0; j <= C->ny; ++j)
            for (int i = 0; i < C->nx; ++i) {
                double s = 0.0;
                for (int dk = 0; dk < 2; ++dk)
                    for (int di = 0; di < 2; ++di) s += *byp(F, 2 * i + di, 2 * j, 2 * k + dk);
                *byp(C, i, j, k) = 0.25 * s;
            }
    for (int k = 0; k <= C->nz; ++k)
        for (int j = 0; j < C->ny; ++j)
            for (int i = 0; i < C->nx; ++i) {
                double s = 0.0;
                for (int dj = 0; dj < 2; ++dj)
                    for (int di = 0; di < 2; ++di) s += *bzp(F, 2 * i + di, 2 * j + dj, 2 * k);
                *bzp(C, i, j, k) = 0.25 * s;
            }
}

/* Sum over the 6 faces of cell (i,j,k): off = sum beta_f u_N (interior),
 * dg = sum beta_f (interior) + sum 2 beta_f (Dirichlet).  Unscaled by h^-2. */
static void cell_terms(const orc_level *L, const double *u, int i, int j, int k, double *off,
                       double *dg) {
    double o = 0.0, d = 0.0, be;
    /* x- */
    be = *bxp(L, i, j, k);
    if (i > 0) { o += be * u[idx(L, i - 1, j, k)]; d += be; }
    else if (L->bc_type[0] == ORC_DIRICHLET) d += 2.0 * be;
    /* x+ */
    be = *bxp(L, i + 1, j, k);
    if (i < L->nx - 1) { o += be * u[idx(L, i + 1, j, k)]; d += be; }
    else if (L->bc_type[1] == ORC_DIRICHLET) d += 2.0 * be;
    /* y- */
    be = *byp(L, i, j, k);
    if (j > 0) { o += be * u[idx(L, i, j - 1, k)]; d += be; }
    else if (L->bc_type[2] == ORC_DIRICHLET) d += 2.0 * be;
    /* y+ */
    be = *byp(L, i, j + 1, k);
    if (j < L->ny - 1) { o += be * u[idx(L, i, j + 1, k)]; d += be; }
    else if (L->bc_type[3] == ORC_DIRICHLET) d += 2.0 * be;
    /* z- */
    be = *bzp(L, i, j, k);
    if (k > 0) { o += be * u[idx(L, i, j, k - 1)]; d += be; }
    else if (L->bc_type[4] == ORC_DIRICHLET) d += 2.0 * be;
    /* z+ */
    be = *bzp(L, i, j, k + 1);
    if (k < L->nz - 1) { o += be * u[idx(L, i, j, k + 1)]; d += be; }
    else if (L->bc_type[5] == ORC_DIRICHLET) d += 2.0 * be;
    *off = o;
    *dg = d;
}

static void level_apply(const orc_level *L, const double *u, double *out) {
    const double ih2 = 1.0 / (L->h * L->h);
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < L->nz; ++k)
        for (int j = 0; j < L->ny; ++j)
            for (int i = 0; i < L->nx; ++i) {
                double o, d;
                cell_terms(L, u, i, j, k, &o, &d);
                size_t p = idx(L, i, j, k);
                out[p] = L->a * u[p] + ih2 * (d * u[p] - o);
            }
}

static void level_residual(const orc_level *L, const double *b, const double *u, double *r) {
    level_apply(L, u, r);
    size_t n = ncell(L);
    for (size_t p = 0; p < n; ++p) r[p] = b[p] - r[p];
}

/* One lexicographic Gauss-Seidel sweep (i fastest, then j, then k). */
static void level_gs(const orc_level *L, const double *b, double *u) {
    const double ih2 = 1.0 / (L->h * L->h);
    for (int k = 0; k < L->nz; ++k)
        for (int j = 0; j < L->ny; ++j)
            for (int i = 0; i < L->nx; ++i) {
                double o, d;
                cell_terms(L, u, i, j, k, &o, &d);
                size_t p = idx(L, i, j, k);
                u[p] = (b[p] + ih2 * o) / (L->a + ih2 * d);
            }
}

static double dot(const double *x, const double *y, size_t n) {
    double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (size_t p = 0; p < n; ++p) s += x[p] * y[p];
    return s;
}

/* Plain conjugate gradients on A u = b from the given u. */
static int level_cg(const orc_level *L, const double *b, double *u, double rtol, int maxit,
                    double *relres) {
    size_t n = ncell(L);
    double *r = (double *)malloc(n * sizeof(double));
    double *p = (double *)malloc(n * sizeof(double));
    double *q = (double *)malloc(n * sizeof(double));
    double bn = sqrt(dot(b, b, n));
    level_residual(L, b, u, r);
    memcpy(p, r, n * sizeof(double));
    double rr = dot(r, r, n);
    int it = 0;
    if (bn == 0.0) bn = 1.0;
    while (it < maxit && sqrt(rr) > rtol * bn) {
        level_apply(L, p, q);
        double alpha = rr / dot(p, q, n);
#pragma omp parallel for schedule(static)
        for (size_t m = 0; m < n; ++m) {
            u[m] += alpha * p[m];
            r[m] -= alpha * q[m];
        }
        double rr_new = dot(r, r, n);
        double beta = rr_new / rr;
        rr = rr_new;
#pragma omp parallel for schedule(static)
        for (size_t m = 0; m < n; ++m) p[m] = r[m] + beta * p[m];
        ++it;
    }
    /* report the true residual, not the recursively updated one */
    level_residual(L, b, u, r);
    *relres = sqrt(dot(r, r, n)) / bn;
    free(r);
    free(p);
    free(q);
    return it;
}

static void restrict_avg(const orc_level *F, const double *r, const orc_level *C, double *bc) {
    for (int k = 0; k < C->nz; ++k)
        for (int j = 0; j < C->ny; ++j)
            for (int i = 0; i < C->nx; ++i) {
                double s = 0.0;
                for (int dk = 0; dk < 2; ++dk)
                    for (int dj = 0; dj < 2; ++dj)
                        for (int di = 0; di < 2; ++di)
                            s += r[idx(F, 2 * i + di, 2 * j + dj, 2 * k + dk)];
                bc[idx(C, i, j, k)] = 0.125 * s;
            }
}

/* Coarse value with ghost reflection: an index one step outside the box on
 * an axis maps to the boundary cell, negated for a Dirichlet face. */
static double coarse_val(const orc_level *C, const double *e, int i, int j, int k) {
    double sgn = 1.0;
    if (i < 0) { i = 0; if (C->bc_type[0] == ORC_DIRICHLET) sgn = -sgn; }
    if (i >= C->nx) { i = C->nx - 1; if (C->bc_type[1] == ORC_DIRICHLET) sgn = -sgn; }
    if (j < 0) { j = 0; if (C->bc_type[2] == ORC_DIRICHLET) sgn = -sgn; }
    if (j >= C->ny) { j = C->ny - 1; if (C->bc_type[3] == ORC_DIRICHLET) sgn = -sgn; }
    if (k < 0) { k = 0; if (C->bc_type[4] == ORC_DIRICHLET) sgn = -sgn; }
    if (k >= C->nz) { k = C->nz - 1; if (C->bc_type[5] == ORC_DIRICHLET) sgn = -sgn; }
    return sgn * e[idx(C, i, j, k)];
}

static void prolong_add(const orc_level *C, const double *e, const orc_level *F, double *u) {
    for (int k = 0; k < F->nz; ++k)
        for (int j = 0; j < F->ny; ++j)
            for (int i = 0; i < F->nx; ++i) {
                int I = i / 2, J = j / 2, K = k / 2;
                int si = (i % 2) ? 1 : -1, sj = (j % 2) ? 1 : -1, sk = (k % 2) ? 1 : -1;
                double v = 0.0;
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b)
                        for (int c = 0; c < 2; ++c) {
                            double w = (a ? 0.25 : 0.75) * (b ? 0.25 : 0.75) * (c ? 0.25 : 0.75);
                            v += w * coarse_val(C, e, I + a * si, J + b * sj, K + c * sk);
                        }
                u[idx(F, i, j, k)] += v;
            }
}

typedef struct {
    int nlev;
    orc_level lev[32];
    double *u[32], *b[32], *r[32];
} orc_hier;

static void level0_coef(orc_level *L, orc_coef C) {
    if (C.bx) {
        memcpy(L->bx, C.bx, (size_t)(L->nx + 1) * L->ny * L->nz * sizeof(double));
        memcpy(L->by, C.by, (size_t)L->nx * (L->ny + 1) * L->nz * sizeof(double));
        memcpy(L->bz, C.bz, (size_t)L->nx * L->ny * (L->nz + 1) * sizeof(double));
    } else {
        level0_faces(L, C.eps);
    }
}

static void hier_build(orc_hier *H, int nx, int ny, int nz, double h, double a, orc_coef coef,
                       const int *bct, int coarsest_max) {
    memset(H, 0, sizeof(*H));
    orc_level *L = &H->lev[0];
    L->nx = nx; L->ny = ny; L->nz = nz; L->h = h; L->a = a;
    memcpy(L->bc_type, bct, 6 * sizeof(int));
    level_alloc(L);
    level0_coef(L, coef);
    H->nlev = 1;
    for (;;) {
        orc_level *F = &H->lev[H->nlev - 1];
        int mx = F->nx > F->ny ? F->nx : F->ny;
        if (F->nz > mx) mx = F->nz;
        if (mx <= coarsest_max) break;
        if (F->nx % 2 || F->ny % 2 || F->nz % 2) break;
        orc_level *C = &H->lev[H->nlev];
        C->nx = F->nx / 2; C->ny = F->ny / 2; C->nz = F->nz / 2;
        C->h = 2.0 * F->h; C->a = F->a;
        memcpy(C->bc_type, F->bc_type, 6 * sizeof(int));
        level_alloc(C);
        coarsen_faces(F, C);
        H->nlev++;
    }
    for (int l = 0; l < H->nlev; ++l) {
        size_t n = ncell(&H->lev[l]);
        H->u[l] = (double *)calloc(n, sizeof(double));
        H->b[l] = (double *)calloc(n, sizeof(double));
        H->r[l] = (double *)calloc(n, sizeof(double));
    }
}

static void hier_free(orc_hier *H) {
    for (int l = 0; l < H->nlev; ++l) {
        level_free(&H->lev[l]);
        free(H->u[l]);
        free(H->b[l]);
        free(H->r[l]);
    }
}

/* V-cycle on level l: u[l] holds the iterate, b[l] the right-hand side. */
static void vcycle(orc_hier *H, int l, int nu1, int nu2) {
    orc_level *L = &H->lev[l];
    if (l == H->nlev - 1) {
        double rr;
        level_cg(L, H->b[l], H->u[l], 1e-14, 10 * (int)ncell(L) + 100, &rr);
        return;
    }
    for (int s = 0; s < nu1; ++s) level_gs(L, H->b[l], H->u[l]);
    level_residual(L, H->b[l], H->u[l], H->r[l]);
    restrict_avg(L, H->r[l], &H->lev[l + 1], H->b[l + 1]);
    memset(H->u[l + 1], 0, ncell(&H->lev[l + 1]) * sizeof(double));
    vcycle(H, l + 1, nu1, nu2);
    prolong_add(&H->lev[l + 1], H->u[l + 1], L, H->u[l]);
    for (int s = 0; s < nu2; ++s) level_gs(L, H->b[l], H->u[l]);
}

/* ---------------------------------------------------------------- API */

static void bc_rhs(const orc_level *L, const double *g, const double *f, double *b) {
    /* b = f + h^-2 sum_Dirichlet 2 beta_b g, beta_b the coefficient of the
     * boundary face (for a cell coefficient: the boundary cell's own) */
    const double ih2 = 1.0 / (L->h * L->h);
    for (int k = 0; k < L->nz; ++k)
        for (int j = 0; j < L->ny; ++j)
            for (int i = 0; i < L->nx; ++i) {
                size_t p = idx(L, i, j, k);
                double s = 0.0;
                if (i == 0 && L->bc_type[0] == ORC_DIRICHLET) s += 2.0 * *bxp(L, 0, j, k) * g[0];
                if (i == L->nx - 1 && L->bc_type[1] == ORC_DIRICHLET) s += 2.0 * *bxp(L, L->nx, j, k) * g[1];
                if (j == 0 && L->bc_type[2] == ORC_DIRICHLET) s += 2.0 * *byp(L, i, 0, k) * g[2];
                if (j == L->ny - 1 && L->bc_type[3] == ORC_DIRICHLET) s += 2.0 * *byp(L, i, L->ny, k) * g[3];
                if (k == 0 && L->bc_type[4] == ORC_DIRICHLET) s += 2.0 * *bzp(L, i, j, 0) * g[4];
                if (k == L->nz - 1 && L->bc_type[5] == ORC_DIRICHLET) s += 2.0 * *bzp(L, i, j, L->nz) * g[5];
                b[p] = f[p] + ih2 * s;
            }
}

static void make_level0(orc_level *L, int nx, int ny, int nz, double h, double a,
                        orc_coef coef, const int *bct) {
    memset(L, 0, sizeof(*L));
    L->nx = nx; L->ny = ny; L->nz = nz; L->h = h; L->a = a;
    memcpy(L->bc_type, bct, 6 * sizeof(int));
    level_alloc(L);
    level0_coef(L, coef);
}

/* Each public routine comes in two forms: with a cell coefficient eps
 * (NULL = 1; faces by harmonic means) and, suffixed _faces, with the face
 * coefficients bx, by, bz given directly. */

static void apply_c(int nx, int ny, int nz, double h, double a, orc_coef C, const int *bct, const double *u,
                    double *out) {
    orc_level L;
    make_level0(&L, nx, ny, nz, h, a, C, bct);
    level_apply(&L, u, out);
    level_free(&L);
}

static void rhs_c(int nx, int ny, int nz, double h, double a, orc_coef C, const int *bct, const double *g,
                  const double *f, double *b) {
    orc_level L;
    make_level0(&L, nx, ny, nz, h, a, C, bct);
    bc_rhs(&L, g, f, b);
    level_free(&L);
}

static double residual_c(int nx, int ny, int nz, double h, double a, orc_coef C, const int *bct,
                         const double *g, const double *f, const double *u, double *r, double *bnorm) {
    orc_level L;
    make_level0(&L, nx, ny, nz, h, a, C, bct);
    size_t n = ncell(&L);
    double *b = (double *)malloc(n * sizeof(double));
    bc_rhs(&L, g, f, b);
    level_residual(&L, b, u, r);
    *bnorm = sqrt(dot(b, b, n));
    double rn = sqrt(dot(r, r, n));
    free(b);
    level_free(&L);
    return rn;
}

static int cg_c(int nx, int ny, int nz, double h, double a, orc_coef C, const int *bct, const double *g,
                const double *f, double *u, double rtol, int maxit, double *relres) {
    orc_level L;
    make_level0(&L, nx, ny, nz, h, a, C, bct);
    size_t n = ncell(&L);
    double *b = (double *)malloc(n * sizeof(double));
    bc_rhs(&L, g, f, b);
    int it = level_cg(&L, b, u, rtol, maxit, relres);
    free(b);
    level_free(&L);
    return it;
}

static int vcycle_solve_c(int nx, int ny, int nz, double h, double a, orc_coef C, const int *bct,
                          const double *g, const double *f, double *u, double rtol, int max_cycles, int nu1,
                          int nu2, int coarsest_max, double *relres, double *history) {
    orc_hier H;
    hier_build(&H, nx, ny, nz, h, a, C, bct, coarsest_max);
    orc_level *L = &H.lev[0];
    size_t n = ncell(L);
    bc_rhs(L, g, f, H.b[0]);
    memcpy(H.u[0], u, n * sizeof(double));
    double bn = sqrt(dot(H.b[0], H.b[0], n));
    if (bn == 0.0) bn = 1.0;
    level_residual(L, H.b[0], H.u[0], H.r[0]);
    double rel = sqrt(dot(H.r[0], H.r[0], n)) / bn;
    int c = 0;
    while (c < max_cycles && rel > rtol) {
        vcycle(&H, 0, nu1, nu2);
        level_residual(L, H.b[0], H.u[0], H.r[0]);
        rel = sqrt(dot(H.r[0], H.r[0], n)) / bn;
        if (history) history[c] = rel;
        ++c;
    }
    memcpy(u, H.u[0], n * sizeof(double));
    *relres = rel;
    hier_free(&H);
    return c;
}

/* Red-black Gauss-Seidel sweeps of the finest-level equation (the paper's
 * smoother, Sec. 2 item (ii)): first every red cell ((i+j+k) even), then
 * every black cell, each set to the value that zeroes its own residual.
 * A red cell's neighbours are all black (and vice versa), so the order
 * inside a colour does not matter. */
static void rbgs_c(int nx, int ny, int nz, double h, double a, orc_coef C, const int *bct, const double *g,
                   const double *f, double *u, int sweeps) {
    orc_level L;
    make_level0(&L, nx, ny, nz, h, a, C, bct);
    size_t n = ncell(&L);
    double *b = (double *)malloc(n * sizeof(double));
    bc_rhs(&L, g, f, b);
    const double ih2 = 1.0 / (h * h);
    for (int s = 0; s < sweeps; ++s)
        for (int colour = 0; colour < 2; ++colour)
            for (int k = 0; k < nz; ++k)
                for (int j = 0; j < ny; ++j)
                    for (int i = 0; i < nx; ++i) {
                        if (((i + j + k) & 1) != colour) continue;
                        double o, d;
                        cell_terms(&L, u, i, j, k, &o, &d);
                        size_t p = idx(&L, i, j, k);
                        u[p] = (b[p] + ih2 * o) / (a + ih2 * d);
                    }
    free(b);
    level_free(&L);
}

/* out = A u (homogeneous boundary values). */
void orc_apply(int nx, int ny, int nz, double h, double a, const double *eps, const int *bct,
               const double *u, double *out) {
    apply_c(nx, ny, nz, h, a, cell_coef(eps), bct, u, out);
}
void orc_apply_faces(int nx, int ny, int nz, double h, double a, const double *bx, const double *by,
                     const double *bz, const int *bct, const double *u, double *out) {
    apply_c(nx, ny, nz, h, a, face_coef(bx, by, bz), bct, u, out);
}

/* b = f + boundary terms of the Dirichlet values g[6]. */
void orc_rhs(int nx, int ny, int nz, double h, double a, const double *eps, const int *bct,
             const double *g, const double *f, double *b) {
    rhs_c(nx, ny, nz, h, a, cell_coef(eps), bct, g, f, b);
}
void orc_rhs_faces(int nx, int ny, int nz, double h, double a, const double *bx, const double *by,
                   const double *bz, const int *bct, const double *g, const double *f, double *b) {
    rhs_c(nx, ny, nz, h, a, face_coef(bx, by, bz), bct, g, f, b);
}

/* Writes r = b - A u and returns ||r||_2; *bnorm = ||b||_2. */
double orc_residual(int nx, int ny, int nz, double h, double a, const double *eps,
                    const int *bct, const double *g, const double *f, const double *u,
                    double *r, double *bnorm) {
    return residual_c(nx, ny, nz, h, a, cell_coef(eps), bct, g, f, u, r, bnorm);
}
double orc_residual_faces(int nx, int ny, int nz, double h, double a, const double *bx, const double *by,
                          const double *bz, const int *bct, const double *g, const double *f, const double *u,
                          double *r, double *bnorm) {
    return residual_c(nx, ny, nz, h, a, face_coef(bx, by, bz), bct, g, f, u, r, bnorm);
}

/* CG from the given u to ||b - A u|| <= rtol ||b||.  Returns iterations. */
int orc_cg(int nx, int ny, int nz, double h, double a, const double *eps, const int *bct,
           const double *g, const double *f, double *u, double rtol, int maxit, double *relres) {
    return cg_c(nx, ny, nz, h, a, cell_coef(eps), bct, g, f, u, rtol, maxit, relres);
}
int orc_cg_faces(int nx, int ny, int nz, double h, double a, const double *bx, const double *by,
                 const double *bz, const int *bct, const double *g, const double *f, double *u, double rtol,
                 int maxit, double *relres) {
    return cg_c(nx, ny, nz, h, a, face_coef(bx, by, bz), bct, g, f, u, rtol, maxit, relres);
}

/* Multigrid V(nu1,nu2) cycles with lexicographic Gauss-Seidel from the given
 * u until ||b - A u|| <= rtol ||b|| or max_cycles.  Coarsening halves every
 * axis while all are even and the largest exceeds coarsest_max; the coarsest
 * level is solved by CG.  Returns cycles; *relres the final relative
 * residual. */
int orc_vcycle_solve(int nx, int ny, int nz, double h, double a, const double *eps,
                     const int *bct, const double *g, const double *f, double *u, double rtol,
                     int max_cycles, int nu1, int nu2, int coarsest_max, double *relres,
                     double *history) {
    return vcycle_solve_c(nx, ny, nz, h, a, cell_coef(eps), bct, g, f, u, rtol, max_cycles, nu1, nu2,
                          coarsest_max, relres, history);
}
int orc_vcycle_solve_faces(int nx, int ny, int nz, double h, double a, const double *bx, const double *by,
                           const double *bz, const int *bct, const double *g, const double *f, double *u,
                           double rtol, int max_cycles, int nu1, int nu2, int coarsest_max, double *relres,
                           double *history) {
    return vcycle_solve_c(nx, ny, nz, h, a, face_coef(bx, by, bz), bct, g, f, u, rtol, max_cycles, nu1, nu2,
                          coarsest_max, relres, history);
}

void orc_rbgs(int nx, int ny, int nz, double h, double a, const double *eps, const int *bct,
              const double *g, const double *f, double *u, int sweeps) {
    rbgs_c(nx, ny, nz, h, a, cell_coef(eps), bct, g, f, u, sweeps);
}
void orc_rbgs_faces(int nx, int ny, int nz, double h, double a, const double *bx, const double *by,
                    const double *bz, const int *bct, const double *g, const double *f, double *u, int sweeps) {
    rbgs_c(nx, ny, nz, h, a, face_coef(bx, by, bz), bct, g, f, u, sweeps);
}

/* Number of levels the V-cycle oracle builds (for reporting). */
int orc_num_levels(int nx, int ny, int nz, int coarsest_max) {
    int n = 1;
    for (;;) {
        int mx = nx > ny ? nx : ny;
        if (nz > mx) mx = nz;
        if (mx <= coarsest_max || nx % 2 || ny % 2 || nz % 2) break;
        nx /= 2; ny /= 2; nz /= 2;
        ++n;
    }
    return n;
}

/* u (2nxc x 2nyc x 2nzc) += P e, the trilinear prolongation of the coarse
 * field e (nxc x nyc x nzc) with the coarse level's face types bct, as one
 * V-cycle applies it to the coarse correction. */
void orc_prolong_add(int nxc, int nyc, int nzc, const int *bct, const double *e, double *u) {
    orc_level C, F;
    memset(&C, 0, sizeof C);
    memset(&F, 0, sizeof F);
    C.nx = nxc; C.ny = nyc; C.nz = nzc;
    F.nx = 2 * nxc; F.ny = 2 * nyc; F.nz = 2 * nzc;
    memcpy(C.bc_type, bct, 6 * sizeof(int));
    memcpy(F.bc_type, bct, 6 * sizeof(int));
    prolong_add(&C, e, &F, u);
}

/* Red-black Gauss-Seidel sweeps of level `level` of the hierarchy that
 * coarsens while every axis is even and the largest exceeds 1 (level 0 =
 * the given grid): the homogeneous correction equation A_l u = b of that
 * level (Dirichlet faces with value 0), with the level's rediscretised
 * coefficients (level 0: harmonic-mean faces of eps; coarser levels: the
 * mean of the four fine faces each coarse face covers).  b and u have the
 * level's dimensions.  Returns the number of levels (u untouched if
 * `level` does not exist). */
int orc_rbgs_level(int nx, int ny, int nz, double h, double a, const double *eps, const int *bct, int level,
                   const double *b, double *u, int sweeps) {
    orc_hier H;
    hier_build(&H, nx, ny, nz, h, a, cell_coef(eps), bct, 1);
    const int nlev = H.nlev;
    if (level >= 0 && level < nlev) {
        const orc_level *L = &H.lev[level];
        const double ih2 = 1.0 / (L->h * L->h);
        for (int s = 0; s < sweeps; ++s)
            for (int colour = 0; colour < 2; ++colour)
                for (int k = 0; k < L->nz; ++k)
                    for (int j = 0; j < L->ny; ++j)
                        for (int i = 0; i < L->nx; ++i) {
                            if (((i + j + k) & 1) != colour) continue;
                            double o, d;
                            cell_terms(L, u, i, j, k, &o, &d);
                            size_t p = idx(L, i, j, k);
                            u[p] = (b[p] + ih2 * o) / (L->a + ih2 * d);
                        }
    }
    hier_free(&H);
    return nlev;
}

/* Threads the oracle's parallel loops use (1 without OpenMP). */
int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
