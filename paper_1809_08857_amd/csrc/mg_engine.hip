// Host driver of the multigrid engine and the C ABI declared in mg.h.
//
// A context owns the level hierarchy of one grid and operator.  mg_solve
// runs V-cycles (MG_FP64) or FP64 iterative refinement around
// low-precision V-cycles (MG_FP32_IR, MG_BF16_IR); every arithmetic step is
// a HIP kernel enqueued on the context's stream, and the host reads back
// one residual norm per cycle to decide convergence.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "mg.h"
#include "mg_engine.h"

namespace mg {

thread_local std::string g_err;

int set_err(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define CK(expr)                                                                                   \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return set_err(MG_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),       \
                           __FILE__, __LINE__);                                                    \
    } while (0)

static void *dalloc(Ctx *c, size_t bytes) {
    void *p = nullptr;
    if (bytes == 0) bytes = 8;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    c->allocs.push_back(p);
    return p;
}

static void dfree(Ctx *c, void *&p) {
    if (!p) return;
    auto it = std::find(c->allocs.begin(), c->allocs.end(), p);
    if (it != c->allocs.end()) c->allocs.erase(it);
    (void)hipFree(p);
    p = nullptr;
}

Geo level_geo(const Ctx *c, int l, bool with_g, bool lowp) {
    const Level &L = c->L[l];
    Geo G;
    G.nx = L.nx;
    G.ny = L.ny;
    G.nz = L.nz;
    G.bcmask = c->bcmask;
    G.h2 = L.h * L.h;
    G.a = lowp ? c->a * c->cscale : c->a;
    G.ah2 = G.a * G.h2;
    G.ih2 = 1.0 / G.h2;
    for (int d = 0; d < 6; ++d) G.g[d] = (with_g && l == 0) ? c->g[d] : 0.0;
    G.cw = l == 0 ? c->corr_w : 1.0;
    return G;
}

Coef level_coef(const Ctx *c, int l, bool lowp) {
    Coef C{};
    if (!c->has_eps) {
        C.mode = COEF_CONST;
        return C;
    }
    if (l == 0 && !c->face0) {
        C.mode = COEF_CELL;
        C.eps = lowp ? c->eps_lp : (const void *)c->eps;
        return C;
    }
    C.mode = c->has_diag ? COEF_FACED : COEF_FACE;
    const Level &L = c->L[l];
    C.dd = c->has_diag ? L.dd : nullptr;
    if (lowp) {
        C.bx = L.lbx;
        C.by = L.lby;
        C.bz = L.lbz;
    } else {
        C.bx = L.fbx;
        C.by = L.fby;
        C.bz = L.fbz;
    }
    return C;
}

void build_tail(const Ctx *c, TailDesc &D, bool with_g) {
    std::memset(&D, 0, sizeof D);
    D.nlev = c->nlev - c->tail;
    D.mode = c->has_diag ? COEF_FACED : (c->has_eps ? COEF_FACE : COEF_CONST);
    D.bcmask = c->bcmask;
    for (int d = 0; d < 6; ++d) D.g[d] = (with_g && c->tail == 0) ? c->g[d] : 0.0;
    D.nu1 = std::max(1, c->d.nu1);
    D.nu2 = std::max(1, c->d.nu2);
    D.ncyc = 1;
    for (int q = 0; q < D.nlev; ++q) {
        const Level &L = c->L[c->tail + q];
        TailLevel &T = D.L[q];
        T.nx = L.nx;
        T.ny = L.ny;
        T.nz = L.nz;
        T.h2 = L.h * L.h;
        T.ah2 = c->a * c->cscale * T.h2;  // cscale = 1 unless the faces are those of the inner operator
        T.bx = L.fbx;
        T.by = L.fby;
        T.bz = L.fbz;
        T.dd = c->has_diag ? L.dd : nullptr;
    }
    const TailLevel &Lc = D.L[D.nlev - 1];
    D.cg_maxit = 2 * Lc.nx * Lc.ny * Lc.nz + 50;
    D.cg_rtol = 1e-13;
    D.stage = 1;
    if (!tail_layout(D)) {  // coefficients too large for LDS: read them from memory
        D.stage = 0;
        tail_layout(D);
    }
}

void set_screening(Ctx *c, double a) {
    c->a = a;
    build_tail(c, c->tails[0], false);
    build_tail(c, c->tails[1], true);
}

// ------------------------------------------------------------ V-cycle

int tile_for(const Ctx *c, const Geo &G, int st, int mode, int l, int *zc) {
    int t = 0, z = 0;
    if (l == 0) {
        t = (st == ST_F64) ? c->tile64 : c->tile_lp;
        z = (st == ST_F64) ? c->zc64 : c->zc_lp;
    }
    if (t <= 0) t = default_tile(G, st, mode);
    if (z <= 0) z = default_zchunk(G, t, st, mode);
    *zc = z;
    return t;
}

// One V-cycle from level l of a view, starting from zero when zero_start
// (otherwise from view[l].u).  The result is in view[l].u afterwards (the
// pointer may have been swapped with view[l].t).  Every kernel returns at
// once when *done is set.
int vcycle(Ctx *c, std::vector<LvView> &V, int l, bool zero_start, const int *done) {
    hipStream_t s = c->stream;
    LvView &W = V[l];
    if (l == c->tail) {
        CK(tail_solve(s, W.st, c->tails[W.st == ST_F64 && W.with_g ? 1 : 0], W.b,
                      zero_start ? nullptr : W.u, W.u, done));
        return MG_OK;
    }
    int zc;
    const int tile = tile_for(c, W.G, W.st, W.C.mode, l, &zc);
    bool zin = zero_start;
    for (int q = 0; q < c->d.nu1; ++q) {
        CK(timed_smooth(c, l, W, zin, tile, zc, done));
        std::swap(W.u, W.t);
        zin = false;
    }
    if (zin) CK(fill_zero(s, W.u, W.n * store_size(W.st), done));
    RrCheck chk;
    chk.done_in = done;
    CK(resid_restrict(s, W.st, W.G, W.C, W.u, W.b, V[l + 1].st, V[l + 1].bw, chk));
    int rc = vcycle(c, V, l + 1, true, done);
    if (rc != MG_OK) return rc;
    CK(prolong_add(s, W.st, W.G, W.u, V[l + 1].st, V[l + 1].G, V[l + 1].u, done));
    for (int q = 0; q < c->d.nu2; ++q) {
        CK(timed_smooth(c, l, W, false, tile, zc, done));
        std::swap(W.u, W.t);
    }
    return MG_OK;
}

void fp64_view(Ctx *c, std::vector<LvView> &V, const double *f, double *x) {
    V.assign(c->tail + 1, LvView{});
    for (int l = 0; l <= c->tail; ++l) {
        LvView &W = V[l];
        W.st = ST_F64;
        W.G = level_geo(c, l, true);
        W.C = level_coef(c, l, false);
        W.n = c->L[l].n;
        W.with_g = (l == 0);
        if (l == 0) {
            W.u = x;
            W.t = c->xalt;
            W.b = f;
            W.fixed_u = true;
        } else {
            W.u = c->L[l].u;
            W.t = c->L[l].t;
            W.b = c->L[l].b;
            W.bw = c->L[l].b;
        }
    }
}

void lowp_view(Ctx *c, std::vector<LvView> &V) {
    V.assign(c->tail + 1, LvView{});
    for (int l = 0; l <= c->tail; ++l) {
        LvView &W = V[l];
        W.st = c->lp_store;
        W.G = level_geo(c, l, false, true);
        W.C = level_coef(c, l, true);
        W.n = c->L[l].n;
        W.u = c->L[l].ul;
        W.t = c->L[l].tl;
        W.b = c->L[l].bl;
        W.bw = c->L[l].bl;
    }
}

static const char *mode_name(int m) {
    return m == COEF_CELL ? "cell-eps" : (m == COEF_FACE ? "face" : (m == COEF_FACED ? "face+diag" : "const"));
}

// Finest-level smoother launch, bracketed by events while timing is on
// (sweeps of a given iterate only: the zero-input variant of a cycle's
// first sweep is another kernel).
hipError_t timed_smooth(Ctx *c, int l, const LvView &W, bool zin, int tile, int zc, const int *done) {
    const bool rec = c->timing && l == 0 && !zin && c->ev_used + 2 <= (int)c->ev.size();
    if (rec) {
        hipError_t e = hipEventRecord(c->ev[c->ev_used], c->stream);
        if (e != hipSuccess) return e;
    }
    hipError_t e = smooth(c->stream, W.st, W.G, W.C, W.u, W.t, W.b, zin, tile, zc, done);
    if (e != hipSuccess || !rec) return e;
    e = hipEventRecord(c->ev[c->ev_used + 1], c->stream);
    if (e != hipSuccess) return e;
    // algorithmic bytes: read u (unless zero), b and eps once, write u once
    const double es = (double)store_size(W.st);
    const int arrays = 1 + 1 + (W.C.mode == COEF_CELL ? 1 : 0) + (is_face_mode(W.C.mode) ? 3 : 0) +
                       (W.C.mode == COEF_FACED ? 1 : 0) + 1;
    c->ev_bytes[c->ev_used / 2] = (double)W.n * es * arrays;
    c->ev_step[c->ev_used / 2] = c->cur_step;
    c->ev_used += 2;
    if (c->t_kernel.empty()) {
        int tx, ty;
        tile_shape(tile, &tx, &ty);
        char buf[160];
        snprintf(buf, sizeof buf, "rbgs_col_k<%s,%s,%d,%d,zero_in=0> (finest-level fused red-black sweep)",
                 W.st == ST_F64 ? "double" : (W.st == ST_F32 ? "float" : "bf16"), mode_name(W.C.mode), tx,
                 ty);
        c->t_kernel = buf;
    }
    return hipSuccess;
}

int timing_flush(Ctx *c, int max_step) {
    if (!c->timing || c->ev_used == 0) return MG_OK;
    CK(hipStreamSynchronize(c->stream));
    for (int q = 0; q + 1 < c->ev_used; q += 2) {
        if (c->ev_step[q / 2] > max_step) continue;
        float ms = 0.f;
        CK(hipEventElapsedTime(&ms, c->ev[q], c->ev[q + 1]));
        c->t_ms += ms;
        c->t_bytes += c->ev_bytes[q / 2];
        c->t_launches++;
    }
    c->ev_used = 0;
    return MG_OK;
}

int read_results(Ctx *c, int n) {
    CK(hipMemcpyAsync(c->h_pin, c->ws.result, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    CK(hipStreamSynchronize(c->stream));
    return MG_OK;
}

int check_grid(const char *who, const mg_desc *d) {
    if (d->nx < 1 || d->ny < 1 || d->nz < 1)
        return set_err(MG_EINVAL, "%s: dimensions must be >= 1 (got %d x %d x %d)", who, d->nx, d->ny, d->nz);
    if ((double)d->nx * d->ny * d->nz > 4.0e9) return set_err(MG_EINVAL, "%s: grid too large", who);
    if ((double)d->nx * d->ny > (double)kMaxPlaneCells)
        return set_err(MG_EINVAL, "%s: an x-y plane may hold at most 2^28 cells", who);
    if (!(d->h > 0.0) || !std::isfinite(d->h)) return set_err(MG_EINVAL, "%s: h must be > 0", who);
    return MG_OK;
}

}  // namespace mg

using namespace mg;

// ====================================================================== C ABI

extern "C" {

void mg_desc_default(mg_desc *d, int nx, int ny, int nz, double h) {
    if (!d) return;
    d->nx = nx;
    d->ny = ny;
    d->nz = nz;
    d->h = h;
    d->precision = MG_FP64;
    d->nu1 = 2;
    d->nu2 = 2;
    d->bottom_max = 16;
    d->max_cycles = 50;
    d->rtol = 1e-10;
}

const char *mg_last_error(void) { return g_err.c_str(); }

int mg_create(const mg_desc *d, void *hip_stream, mg_ctx **out) {
    if (out) *out = nullptr;
    if (!d || !out) return set_err(MG_EINVAL, "mg_create: null argument");
    if (int rc = check_grid("mg_create", d)) return rc;
    if (d->precision < MG_FP64 || d->precision > MG_BF16_IR)
        return set_err(MG_EINVAL, "mg_create: unknown precision %d", d->precision);
    if (d->nu1 < 0 || d->nu2 < 0 || d->nu1 > 8 || d->nu2 > 8 || d->nu1 + d->nu2 < 1)
        return set_err(MG_EINVAL, "mg_create: nu1, nu2 must be in 0..8 with nu1 + nu2 >= 1");
    if (d->bottom_max < 2 || d->bottom_max > 16)
        return set_err(MG_EINVAL, "mg_create: bottom_max must be in 2..16");
    if (d->max_cycles < 1) return set_err(MG_EINVAL, "mg_create: max_cycles must be >= 1");
    if (!(d->rtol > 0.0) || !(d->rtol < 1.0)) return set_err(MG_EINVAL, "mg_create: rtol must be in (0,1)");

    static std::atomic<unsigned long> next_uid{1};
    Ctx *c = new Ctx();
    c->uid = next_uid++;
    c->d = *d;
    c->stream = (hipStream_t)hip_stream;
    c->lp_store = d->precision == MG_FP32_IR ? ST_F32 : (d->precision == MG_BF16_IR ? ST_BF16 : -1);
    // hierarchy: halve every axis while all are even and the largest exceeds 1
    int nx = d->nx, ny = d->ny, nz = d->nz;
    double h = d->h;
    c->nlev = 0;
    c->tail = -1;
    for (;;) {
        if (c->nlev >= kMaxLevels) break;
        Level &L = c->L[c->nlev];
        L.nx = nx;
        L.ny = ny;
        L.nz = nz;
        L.n = (size_t)nx * ny * nz;
        L.h = h;
        const int mx = std::max(nx, std::max(ny, nz));
        if (c->tail < 0 && mx <= d->bottom_max) c->tail = c->nlev;
        c->nlev++;
        if (nx % 2 || ny % 2 || nz % 2 || mx <= 1) break;
        nx /= 2;
        ny /= 2;
        nz /= 2;
        h *= 2.0;
    }
    if (c->tail < 0) {
        delete c;
        return set_err(MG_EINVAL,
                       "mg_create: %d x %d x %d cannot be coarsened to a grid with every axis <= "
                       "bottom_max = %d (each axis must be m * 2^k with the same k)",
                       d->nx, d->ny, d->nz, d->bottom_max);
    }
    if (c->nlev - c->tail > kTailMaxLevels) {
        delete c;
        return set_err(MG_EINVAL, "mg_create: too many bottom levels");
    }
    TailDesc probe;
    build_tail(c, probe, false);
    if (!tail_layout(probe)) {
        delete c;
        return set_err(MG_EINVAL, "mg_create: bottom grid does not fit the bottom solver");
    }
    // buffers
    bool ok = true;
    const size_t n0 = c->L[0].n;
    c->xalt = (double *)dalloc(c, n0 * 8);
    ok &= c->xalt != nullptr;
    // work arrays on every level: the bottom solver may start below the
    // level chosen here (mg_set_coeffs moves it down when the staged
    // coefficients of variable-permittivity operators do not fit in LDS)
    c->tail0 = c->tail;
    for (int l = 1; l < c->nlev; ++l) {
        Level &L = c->L[l];
        L.u = (double *)dalloc(c, L.n * 8);
        L.t = (double *)dalloc(c, L.n * 8);
        L.b = (double *)dalloc(c, L.n * 8);
        ok &= L.u && L.t && L.b;
    }
    if (c->lp_store >= 0) {
        const size_t es = store_size(c->lp_store);
        for (int l = 0; l < c->nlev; ++l) {
            Level &L = c->L[l];
            L.ul = dalloc(c, L.n * es);
            L.tl = dalloc(c, L.n * es);
            L.bl = dalloc(c, L.n * es);
            ok &= L.ul && L.tl && L.bl;
        }
    }
    c->d_done = (int *)dalloc(c, sizeof(int) * 4);
    ok &= c->d_done != nullptr;
    for (int q = 0; q < 2 && ok; ++q) ok &= hipEventCreateWithFlags(&c->ev_cyc[q], hipEventDisableTiming) == hipSuccess;
    c->ws.partials = (double *)dalloc(c, sizeof(double) * kRedSlots * kMaxRedBlocks * 2);
    c->ws.result = (double *)dalloc(c, sizeof(double) * kRedSlots);
    ok &= c->ws.partials && c->ws.result;
    if (ok && hipHostMalloc((void **)&c->h_pin, sizeof(double) * kRedSlots, hipHostMallocDefault) !=
                  hipSuccess)
        ok = false;
    if (!ok) {
        mg_destroy(c);
        return set_err(MG_ENOMEM, "mg_create: device allocation failed");
    }
    if (hipStreamSynchronize(c->stream) != hipSuccess) {
        mg_destroy(c);
        return set_err(MG_EDEVICE, "mg_create: initialisation failed");
    }
    *out = c;
    return MG_OK;
}

int mg_destroy(mg_ctx *c) {
    if (!c) return MG_OK;
    (void)hipStreamSynchronize(c->stream);
    batch_release(c);
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    for (int q = 0; q < 2; ++q)
        if (c->ev_cyc[q]) (void)hipEventDestroy(c->ev_cyc[q]);
    c->ev.clear();
    for (void *p : c->allocs) (void)hipFree(p);
    c->allocs.clear();
    if (c->h_pin) (void)hipHostFree(c->h_pin);
    delete c;
    return MG_OK;
}

}  // extern "C"

namespace mg {

// Validates a and the face conditions of an operator; *mask gets the
// Dirichlet faces.
int parse_operator(const char *who, double a, const mg_bcs *bc, int *mask) {
    if (!(a >= 0.0) || !std::isfinite(a)) return set_err(MG_EINVAL, "%s: a must be finite and >= 0", who);
    int m = 0;
    for (int f = 0; f < 6; ++f) {
        if (bc->type[f] != MG_BC_DIRICHLET && bc->type[f] != MG_BC_NEUMANN)
            return set_err(MG_EINVAL, "%s: unknown boundary type %d on face %d", who, bc->type[f], f);
        if (bc->type[f] == MG_BC_DIRICHLET) {
            if (!std::isfinite(bc->value[f]))
                return set_err(MG_EINVAL, "%s: non-finite boundary value on face %d", who, f);
            m |= 1 << f;
        }
    }
    if (a == 0.0 && m == 0) return set_err(MG_EINVAL, "%s: singular operator (a = 0 and no Dirichlet face)", who);
    *mask = m;
    return MG_OK;
}

static size_t nfaces_x(const Level &L) { return (size_t)(L.nx + 1) * L.ny * L.nz; }
static size_t nfaces_y(const Level &L) { return (size_t)L.nx * (L.ny + 1) * L.nz; }
static size_t nfaces_z(const Level &L) { return (size_t)L.nx * L.ny * (L.nz + 1); }

// FP64 face arrays on every level (level 0 serves the coarsening, and the
// bottom solver when it starts there).
static int alloc_faces(Ctx *c, const char *who) {
    for (int l = 0; l < c->nlev; ++l) {
        Level &L = c->L[l];
        if (!L.fbx) {
            L.fbx = (double *)dalloc(c, nfaces_x(L) * 8);
            L.fby = (double *)dalloc(c, nfaces_y(L) * 8);
            L.fbz = (double *)dalloc(c, nfaces_z(L) * 8);
            if (!L.fbx || !L.fby || !L.fbz) return set_err(MG_ENOMEM, "%s: allocation failed", who);
        }
    }
    return MG_OK;
}

// Coarse face coefficients of levels 1.. from level 0's.
static int coarsen_levels(Ctx *c) {
    for (int l = 1; l < c->nlev; ++l) {
        Level &L = c->L[l];
        const Level &F = c->L[l - 1];
        CK(coarsen_faces(c->stream, level_geo(c, l - 1, false), F.fbx, F.fby, F.fbz, level_geo(c, l, false), L.fbx,
                         L.fby, L.fbz));
    }
    return MG_OK;
}

// Bottom level of a variable-coefficient operator: the first whose staged
// coefficients fit in LDS.
static void choose_bottom(Ctx *c) {
    c->tail = c->tail0;
    for (;;) {
        TailDesc probe;
        build_tail(c, probe, false);
        if (probe.stage || c->tail == c->nlev - 1) break;
        c->tail++;
    }
}

// Common end of the set-up calls: scalar data, bottom descriptors, flags.
static int finish_operator(Ctx *c, double a, int mask, const mg_bcs *bc) {
    c->bcmask = mask;
    for (int f = 0; f < 6; ++f) c->g[f] = (mask >> f & 1) ? bc->value[f] : 0.0;
    set_screening(c, a);
    CK(hipStreamSynchronize(c->stream));
    c->coeffs = true;
    c->version++;
    return MG_OK;
}

}  // namespace mg

extern "C" {

int mg_set_coeffs(mg_ctx *c, const double *eps_dev, double a, const mg_bcs *bc) {
    if (!c || !bc) return set_err(MG_EINVAL, "mg_set_coeffs: null argument");
    int mask = 0, rc = parse_operator("mg_set_coeffs", a, bc, &mask);
    if (rc) return rc;
    hipStream_t s = c->stream;
    const size_t n0 = c->L[0].n;
    c->coeffs = false;
    c->face0 = false;
    c->has_diag = false;
    if (eps_dev) {
        if (!c->eps) {
            c->eps = (double *)dalloc(c, n0 * 8);
            if (!c->eps) return set_err(MG_ENOMEM, "mg_set_coeffs: allocation failed");
        }
        CK(hipMemcpyAsync(c->eps, eps_dev, n0 * 8, hipMemcpyDeviceToDevice, s));
        CK(count_bad(s, c->eps, n0, c->ws, 0));
        if ((rc = read_results(c, 1))) return rc;
        if (c->h_pin[0] != 0.0)
            return set_err(MG_EINVAL, "mg_set_coeffs: %.0f coefficient entries are not in (0, 1e100]",
                           c->h_pin[0]);
        if ((rc = alloc_faces(c, "mg_set_coeffs"))) return rc;
        CK(faces_from_cell(s, level_geo(c, 0, false), c->eps, c->L[0].fbx, c->L[0].fby, c->L[0].fbz));
        if ((rc = coarsen_levels(c))) return rc;
        c->has_eps = true;
        choose_bottom(c);
        c->cscale = 1.0;
        if (c->lp_store >= 0) {
            // The inner cycle runs on eps * cscale with cscale = 2^-m, m the
            // mean binary exponent of the largest and smallest coefficient,
            // so that its FP32 coefficients lie in [2^-35, 2^35]: harmonic
            // means neither overflow nor underflow there, and the Dirichlet
            // coefficient of the FP32 sweeps dominates them.  The scale is a
            // power of two, so every rounding of the inner cycle is the same
            // as without it.  The inner cycle's correction is multiplied by
            // cscale on its way back (ir_update_resid).
            CK(minmax(s, c->eps, n0, c->ws, 2));
            if ((rc = read_results(c, 4))) return rc;
            int emax, emin;
            (void)std::frexp(c->h_pin[2], &emax);
            (void)std::frexp(c->h_pin[3], &emin);
            if (emax - emin > 70)
                return set_err(MG_EINVAL,
                               "mg_set_coeffs: coefficients from %g to %g span more than 2^70, the range of "
                               "the FP32/BF16 inner cycle (use MG_FP64)", c->h_pin[3], c->h_pin[2]);
            const int m = (emax + emin) / 2;
            c->cscale = std::ldexp(1.0, -m);
            if (a * c->cscale > 0x1p100)
                return set_err(MG_EINVAL, "mg_set_coeffs: a = %g is too large against the coefficients for the "
                                          "FP32/BF16 inner cycle (use MG_FP64)", a);
            // the FP64 faces of a mixed-precision context serve only the
            // inner cycle (its bottom solve and its FP32 copies): scale them
            if (c->cscale != 1.0)
                for (int l = 0; l < c->nlev; ++l) {
                    Level &L = c->L[l];
                    CK(scale_f64(s, L.fbx, nfaces_x(L), c->cscale));
                    CK(scale_f64(s, L.fby, nfaces_y(L), c->cscale));
                    CK(scale_f64(s, L.fbz, nfaces_z(L), c->cscale));
                }
            // coefficients of the inner cycle: FP32 for both FP32 and BF16
            // fields (BF16 coefficients perturb the inner operator enough to
            // cost outer steps)
            const int cst = ST_F32;
            const size_t es = store_size(cst);
            if (!c->eps_lp) c->eps_lp = dalloc(c, n0 * es);
            if (!c->eps_lp) return set_err(MG_ENOMEM, "mg_set_coeffs: allocation failed");
            CK(convert(s, c->eps, cst, c->eps_lp, n0, c->cscale));
            for (int l = 1; l < c->tail; ++l) {
                Level &L = c->L[l];
                if (!L.lbx) {
                    L.lbx = dalloc(c, nfaces_x(L) * es);
                    L.lby = dalloc(c, nfaces_y(L) * es);
                    L.lbz = dalloc(c, nfaces_z(L) * es);
                    if (!L.lbx || !L.lby || !L.lbz) return set_err(MG_ENOMEM, "mg_set_coeffs: allocation failed");
                }
                CK(convert(s, L.fbx, cst, L.lbx, nfaces_x(L)));
                CK(convert(s, L.fby, cst, L.lby, nfaces_y(L)));
                CK(convert(s, L.fbz, cst, L.lbz, nfaces_z(L)));
            }
        }
    } else {
        c->has_eps = false;
        c->tail = c->tail0;
        c->cscale = 1.0;
        if (c->lp_store >= 0 && a > 0x1p100)
            return set_err(MG_EINVAL, "mg_set_coeffs: a = %g is too large for the FP32/BF16 inner cycle "
                                      "(use MG_FP64)", a);
    }
    return finish_operator(c, a, mask, bc);
}

static int set_face_impl(const char *who, mg_ctx *c, const double *bx_dev, const double *by_dev,
                         const double *bz_dev, const double *d_dev, double a, const mg_bcs *bc) {
    if (!c || !bc || !bx_dev || !by_dev || !bz_dev) return set_err(MG_EINVAL, "%s: null argument", who);
    if (c->lp_store >= 0) return set_err(MG_EINVAL, "%s: face coefficients need an MG_FP64 context", who);
    int mask = 0, rc = parse_operator(who, a, bc, &mask);
    if (rc) return rc;
    hipStream_t s = c->stream;
    c->coeffs = false;
    c->face0 = false;
    c->has_diag = false;
    if ((rc = alloc_faces(c, who))) return rc;
    Level &L0 = c->L[0];
    CK(hipMemcpyAsync(L0.fbx, bx_dev, nfaces_x(L0) * 8, hipMemcpyDeviceToDevice, s));
    CK(hipMemcpyAsync(L0.fby, by_dev, nfaces_y(L0) * 8, hipMemcpyDeviceToDevice, s));
    CK(hipMemcpyAsync(L0.fbz, bz_dev, nfaces_z(L0) * 8, hipMemcpyDeviceToDevice, s));
    double bad = 0.0;
    const double *arrs[3] = {L0.fbx, L0.fby, L0.fbz};
    const size_t ns[3] = {nfaces_x(L0), nfaces_y(L0), nfaces_z(L0)};
    for (int q = 0; q < 3; ++q) {
        // with a diagonal, faces may vanish (a cut-cell aperture of 0)
        if (d_dev) CK(count_outside(s, arrs[q], ns[q], 0.0, kMaxCellCoef, c->ws, 0));
        else CK(count_bad(s, arrs[q], ns[q], c->ws, 0));
        if ((rc = read_results(c, 1))) return rc;
        bad += c->h_pin[0];
    }
    if (bad != 0.0)
        return set_err(MG_EINVAL, "%s: %.0f face coefficients are not in %s1e100]", who, bad, d_dev ? "[0, " : "(0, ");
    if ((rc = coarsen_levels(c))) return rc;
    if (d_dev) {
        for (int l = 0; l < c->nlev; ++l)
            if (!c->L[l].dd && !(c->L[l].dd = (double *)dalloc(c, c->L[l].n * 8)))
                return set_err(MG_ENOMEM, "%s: allocation failed", who);
        CK(hipMemcpyAsync(L0.dd, d_dev, L0.n * 8, hipMemcpyDeviceToDevice, s));
        CK(count_outside(s, L0.dd, L0.n, 0.0, kMaxCellCoef, c->ws, 0));
        if ((rc = read_results(c, 1))) return rc;
        if (c->h_pin[0] != 0.0)
            return set_err(MG_EINVAL, "%s: %.0f diagonal entries are not in [0, 1e100]", who, c->h_pin[0]);
        for (int l = 1; l < c->nlev; ++l)
            CK(coarsen_cells(s, level_geo(c, l - 1, false), c->L[l - 1].dd, level_geo(c, l, false), c->L[l].dd));
        // every cell of the finest level needs a positive diagonal
        Geo G0 = level_geo(c, 0, false);
        G0.bcmask = mask;
        G0.a = a;
        CK(count_singular(s, G0, L0.fbx, L0.fby, L0.fbz, L0.dd, c->ws, 0));
        if ((rc = read_results(c, 1))) return rc;
        if (c->h_pin[0] != 0.0)
            return set_err(MG_EINVAL, "%s: %.0f cells have no positive diagonal (a + d + faces)", who, c->h_pin[0]);
        c->has_diag = true;
    }
    c->has_eps = true;
    c->face0 = true;
    c->cscale = 1.0;
    choose_bottom(c);
    return finish_operator(c, a, mask, bc);
}

int mg_set_face_coeffs(mg_ctx *c, const double *bx_dev, const double *by_dev, const double *bz_dev, double a,
                       const mg_bcs *bc) {
    return set_face_impl("mg_set_face_coeffs", c, bx_dev, by_dev, bz_dev, nullptr, a, bc);
}

int mg_set_face_coeffs_diag(mg_ctx *c, const double *bx_dev, const double *by_dev, const double *bz_dev,
                            const double *d_dev, double a, const mg_bcs *bc) {
    if (!d_dev) return set_err(MG_EINVAL, "mg_set_face_coeffs_diag: null argument");
    return set_face_impl("mg_set_face_coeffs_diag", c, bx_dev, by_dev, bz_dev, d_dev, a, bc);
}

// Result slots of the reduction workspace used by a solve.
enum { SLOT_R0 = 0, SLOT_B = 1, SLOT_CYC = 2 /* and 3, alternating */ };

static int solve_impl(Ctx *c, const double *f, double *x, unsigned flags, mg_stats *st) {
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = c->stream;
    const size_t n0 = c->L[0].n;
    mg_stats S{};
    const Geo G0 = level_geo(c, 0, true);
    const Coef C0 = level_coef(c, 0, false);
    int *done = c->d_done;
    int rc;
    // ||b|| and the residual of the starting iterate
    // A guess is screened at its first convergence test, after the nu1
    // pre-smoothing sweeps that open every cycle (they remove the
    // cell-scale noise that the operator would otherwise magnify), against
    // the residual of the zero guess, ||b||.  Without a multigrid hierarchy
    // or pre-smoothing the raw residual is compared.
    const bool screen = (flags & MG_GUESS) && c->tail > 0 && c->d.nu1 > 0;
    const bool raw_guess = (flags & MG_GUESS) && !screen;
    if (!(flags & MG_GUESS)) CK(fill_zero(s, x, n0 * 8));
    CK(fill_zero(s, done, sizeof(int)));
    if (raw_guess) {
        CK(norm2_resid(s, ST_F64, G0, C0, x, f, c->ws, SLOT_R0, SLOT_B));
    } else {
        // zero start: ||b - A 0|| = ||b||; a screened guess is tested later
        CK(norm2_b(s, G0, C0, f, c->ws, SLOT_B));
    }
    if ((rc = read_results(c, 2))) return rc;
    const double bn = std::sqrt(c->h_pin[SLOT_B]);
    double rn = raw_guess ? std::sqrt(c->h_pin[SLOT_R0]) : bn;
    if (!std::isfinite(bn) || !std::isfinite(rn))
        return set_err(MG_EINVAL, "mg_solve: right-hand side or initial guess is not finite");
    if (bn == 0.0) {
        CK(fill_zero(s, x, n0 * 8));
        CK(hipStreamSynchronize(s));
        if (st) *st = S;
        return MG_OK;
    }
    if (raw_guess && rn > bn) {
        CK(fill_zero(s, x, n0 * 8));
        S.fell_back = 1;
        rn = bn;
    }
    S.rel_res0 = rn / bn;
    const double rtol = c->d.rtol;
    if (!screen && S.rel_res0 <= rtol) {
        CK(hipStreamSynchronize(s));
        S.rel_res = S.rel_res0;
        if (st) *st = S;
        return MG_OK;
    }
    RrCheck chk;
    chk.ws = c->ws;
    chk.ref_slot = SLOT_B;
    chk.rtol2 = rtol * rtol;
    chk.done_out = done;
    chk.done_in = done;

    // The solve is a pipeline of steps c = 0, 1, ...: check(c) produces the
    // residual norm of the current iterate (and sets *done when it meets the
    // tolerance); advance(c) performs one more cycle.  check(c+1) and
    // advance(c) are enqueued before the host reads the norm of check(c), so
    // the GPU never waits for the host; once *done is set every later kernel
    // returns at once.
    std::vector<LvView> V;
    const bool lowp = c->lp_store >= 0;
    // scale of the first residual cast to the inner storage type (from ||b||;
    // later passes take theirs from the previous residual on the device)
    const double sc0 = cast_scale_rms(bn / std::sqrt((double)n0));
    double *cur = x, *oth = c->xalt;  // FP64 iterate and its spare buffer
    if (lowp) lowp_view(c, V);
    else fp64_view(c, V, f, x);
    auto check = [&](int cyc) -> int {
        c->cur_step = 2 * cyc;
        chk.slot = SLOT_CYC + (cyc & 1);
        if (lowp) {
            // FP64 residual of the starting iterate, cast into the inner
            // right-hand side (later steps get it from advance())
            if (cyc == 0)
                CK(ir_update_resid(s, G0, C0, cur, nullptr, nullptr, f, c->lp_store, V[0].bw, chk, sc0,
                                   c->cscale));
        } else if (c->tail == 0) {
            CK(norm2_resid(s, ST_F64, G0, C0, cur, f, c->ws, chk.slot, -1, &chk));
        } else {
            // level-0 pre-smoothing, then residual + restriction with the norm
            LvView &W = V[0];
            W.u = cur;
            W.t = oth;
            int zc;
            const int tile = tile_for(c, W.G, W.st, W.C.mode, 0, &zc);
            for (int q = 0; q < c->d.nu1; ++q) {
                CK(timed_smooth(c, 0, W, false, tile, zc, done));
                std::swap(W.u, W.t);
            }
            cur = (double *)W.u;
            oth = (double *)W.t;
            CK(resid_restrict(s, ST_F64, W.G, W.C, W.u, W.b, V[1].st, V[1].bw, chk));
        }
        CK(hipMemcpyAsync(c->h_pin + chk.slot, c->ws.result + chk.slot, sizeof(double),
                          hipMemcpyDeviceToHost, s));
        CK(hipEventRecord(c->ev_cyc[cyc & 1], s));
        return MG_OK;
    };
    auto advance = [&](int cyc) -> int {
        c->cur_step = 2 * cyc + 1;
        if (lowp) {
            // inner low-precision V-cycle on A e = r, then x += e (the check
            // of the next step computes the new residual from x and e)
            int r = vcycle(c, V, 0, true, done);
            if (r) return r;
            RrCheck k2 = chk;
            k2.slot = SLOT_CYC + ((cyc + 1) & 1);
            CK(ir_update_resid(s, G0, C0, cur, V[0].u, oth, f, c->lp_store, V[0].bw, k2, 0.0, c->cscale));
            std::swap(cur, oth);
        } else if (c->tail == 0) {
            CK(tail_solve(s, ST_F64, c->tails[1], f, cur, cur, done));
        } else {
            // coarse correction of the restricted residual, then post-smoothing
            LvView &W = V[0];
            int r = vcycle(c, V, 1, true, done);
            if (r) return r;
            CK(prolong_add(s, ST_F64, W.G, cur, ST_F64, V[1].G, V[1].u, done));
            W.u = cur;
            W.t = oth;
            int zc;
            const int tile = tile_for(c, W.G, W.st, W.C.mode, 0, &zc);
            for (int q = 0; q < c->d.nu2; ++q) {
                CK(timed_smooth(c, 0, W, false, tile, zc, done));
                std::swap(W.u, W.t);
            }
            cur = (double *)W.u;
            oth = (double *)W.t;
        }
        return MG_OK;
    };

    if (screen && lowp) {
        // the FP64 pre-smoothing of the guess (the low-precision cycles
        // start from a residual)
        int zc;
        const int tile = tile_for(c, G0, ST_F64, C0.mode, 0, &zc);
        for (int q = 0; q < c->d.nu1; ++q) {
            CK(smooth(s, ST_F64, G0, C0, cur, oth, f, false, tile, zc));
            std::swap(cur, oth);
        }
    }
    if ((rc = check(0))) return rc;
    double *chk0 = cur;  // the iterate check(0) measures
    // With a guess, the first cycle from it is enqueued before the host
    // reads the screen (as every later cycle is enqueued before the host
    // reads the previous norm), so the GPU does not wait for the host.  A
    // fallback discards it: the zero start's kernels follow it on the stream.
    bool spec = false;
    if (screen) {
        if ((rc = advance(0))) return rc;
        if ((rc = check(1))) return rc;
        spec = true;
        CK(hipEventSynchronize(c->ev_cyc[0]));
        const double rel_s = std::sqrt(c->h_pin[SLOT_CYC]) / bn;
        if (!(rel_s <= 1.0)) {  // worse than the zero guess (or not finite): start from zero
            CK(fill_zero(s, x, n0 * 8));
            CK(fill_zero(s, done, sizeof(int)));
            cur = x;
            oth = c->xalt;
            S.fell_back = 1;
            S.rel_res0 = 1.0;
            if ((rc = check(0))) return rc;
            chk0 = cur;
            spec = false;
        } else {
            S.rel_res0 = rel_s;
        }
    }
    double *at_check[2] = {chk0, spec ? cur : nullptr};
    DivergenceWatch watch;
    int cycles = 0;
    double rel = S.rel_res0;
    double *final_x = cur;
    bool converged = false;
    for (int cyc = 0;; ++cyc) {
        if (cyc < c->d.max_cycles && !(spec && cyc == 0)) {
            if ((rc = advance(cyc))) return rc;
            if ((rc = check(cyc + 1))) return rc;
            at_check[(cyc + 1) & 1] = cur;
        }
        CK(hipEventSynchronize(c->ev_cyc[cyc & 1]));
        rel = std::sqrt(c->h_pin[SLOT_CYC + (cyc & 1)]) / bn;
        final_x = at_check[cyc & 1];
        cycles = cyc;
        if (rel <= rtol) {
            converged = true;
            break;
        }
        if (cyc >= c->d.max_cycles) break;
        if (watch.diverged(rel, S.rel_res0)) {
            CK(hipStreamSynchronize(s));
            S.cycles = cycles;
            S.rel_res = rel;
            if (st) *st = S;
            return set_err(MG_EDIVERGED, "mg_solve: residual diverged (%g) after %d cycles", rel, cycles);
        }
    }
    // the iterate that passed the test may sit in the spare buffer
    if (final_x != x) CK(copy_f64(s, final_x, x, n0));
    CK(hipStreamSynchronize(s));
    c->cur_step = -1;
    if ((rc = timing_flush(c, 2 * cycles))) return rc;
    S.cycles = cycles;
    S.rel_res = rel;
    S.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (st) *st = S;
    return converged ? MG_OK : MG_NOT_CONVERGED;
}

int mg_solve(mg_ctx *c, const double *f_dev, double *x_dev, unsigned flags, mg_stats *st) {
    if (!c || !f_dev || !x_dev) return set_err(MG_EINVAL, "mg_solve: null argument");
    if (!c->coeffs) return set_err(MG_EINVAL, "mg_solve: mg_set_coeffs has not succeeded");
    if (flags & ~(unsigned)MG_GUESS) return set_err(MG_EINVAL, "mg_solve: unknown flags 0x%x", flags);
    return solve_impl(c, f_dev, x_dev, flags, st);
}

int mg_apply(mg_ctx *c, double alpha, double beta, const double *x_dev, double *y_dev) {
    if (!c || !x_dev || !y_dev) return set_err(MG_EINVAL, "mg_apply: null argument");
    if (!c->coeffs) return set_err(MG_EINVAL, "mg_apply: mg_set_coeffs has not succeeded");
    if (x_dev == y_dev) return set_err(MG_EINVAL, "mg_apply: x and y must not be the same array");
    if (!std::isfinite(alpha) || !std::isfinite(beta)) return set_err(MG_EINVAL, "mg_apply: alpha, beta not finite");
    CK(apply_op(c->stream, level_geo(c, 0, false), level_coef(c, 0, false), alpha, beta, x_dev, y_dev));
    CK(hipStreamSynchronize(c->stream));
    return MG_OK;
}

int mg_tga_step(mg_ctx *c, double dt, const double *n_dev, double *out_dev, unsigned flags, mg_stats *st) {
    if (!c || !n_dev || !out_dev) return set_err(MG_EINVAL, "mg_tga_step: null argument");
    if (!c->coeffs) return set_err(MG_EINVAL, "mg_tga_step: mg_set_coeffs has not succeeded");
    if (n_dev == out_dev) return set_err(MG_EINVAL, "mg_tga_step: n and out must not be the same array");
    if (!(dt > 0.0) || !std::isfinite(dt)) return set_err(MG_EINVAL, "mg_tga_step: dt must be finite and > 0");
    if (c->bcmask != 0) return set_err(MG_EINVAL, "mg_tga_step: the diffusion operator needs zero flux on every face");
    if (flags & ~(unsigned)MG_GUESS) return set_err(MG_EINVAL, "mg_tga_step: unknown flags 0x%x", flags);
    const size_t n0 = c->L[0].n;
    if (!c->work) {
        c->work = (double *)dalloc(c, n0 * 8);
        if (!c->work) return set_err(MG_ENOMEM, "mg_tga_step: allocation failed");
    }
    // Twizell-Gumel-Arigu coefficients: q = 2 - sqrt(2) - 1e-6, r = sqrt(q^2 - 4q + 2)
    const double q = 2.0 - std::sqrt(2.0) - 1e-6, r = std::sqrt(q * q - 4.0 * q + 2.0);
    const double mu1 = 0.5 * (q - r) * dt, mu2 = 0.5 * (q + r) * dt, mu3 = (1.0 - q) * dt;
    const double a_keep = c->a;
    hipStream_t s = c->stream;
    const Coef C0 = level_coef(c, 0, false);
    mg_stats S[2] = {};
    int rc, worst = MG_OK;
    // (I - mu1 L) y = (I + mu3 L) n, as (1/mu1) y - div(D grad y) = rhs / mu1.  With
    // A the context's operator at a = 1/mu1, L n = a n - A n, so
    // rhs / mu1 = ((1 + mu3 a) n - mu3 A n) / mu1.
    set_screening(c, 1.0 / mu1);
    CK(apply_op(s, level_geo(c, 0, false), C0, (1.0 + mu3 * c->a) / mu1, -mu3 / mu1, n_dev, c->work));
    if (flags & MG_GUESS) CK(copy_f64(s, n_dev, out_dev, n0));  // n as the first guess of y
    rc = solve_impl(c, c->work, out_dev, flags, &S[0]);
    if (rc >= 0) {
        worst = rc;
        // (I - mu2 L) n_new = y, as (1/mu2) n_new - div(D grad n_new) = y / mu2 (y is the guess)
        set_screening(c, 1.0 / mu2);
        rc = MG_OK;
        hipError_t e = apply_op(s, level_geo(c, 0, false), C0, 1.0 / mu2, 0.0, out_dev, c->work);
        if (e != hipSuccess) rc = set_err(MG_EDEVICE, "mg_tga_step: %s", hipGetErrorString(e));
        if (rc == MG_OK) rc = solve_impl(c, c->work, out_dev, flags, &S[1]);
        if (rc > worst) worst = rc;
    }
    set_screening(c, a_keep);
    if (st) {
        st[0] = S[0];
        st[1] = S[1];
    }
    return rc < 0 ? rc : worst;
}

int mg_field(mg_ctx *c, const double *phi_dev, const double *sigma_dev, double eps0, double *ex_dev,
             double *ey_dev, double *ez_dev, double *emax, double *jmax, double *dt_e) {
    if (!c || !phi_dev) return set_err(MG_EINVAL, "mg_field: null argument");
    if (!c->coeffs) return set_err(MG_EINVAL, "mg_field: mg_set_coeffs has not succeeded");
    if (!(eps0 > 0.0) || !std::isfinite(eps0)) return set_err(MG_EINVAL, "mg_field: eps0 must be finite and > 0");
    CK(field(c->stream, level_geo(c, 0, true), c->L[0].h, phi_dev, sigma_dev, ex_dev, ey_dev, ez_dev, c->ws, 2));
    int rc = read_results(c, 4);
    if (rc) return rc;
    const double me = c->h_pin[2], mj = c->h_pin[3];
    if (emax) *emax = me;
    if (jmax) *jmax = mj;
    if (dt_e) *dt_e = mj > 0.0 ? eps0 * me / mj : HUGE_VAL;
    return MG_OK;
}

int mg_relaxation_substeps(double dt_fine, double dt_e, double alpha, int *m) {
    if (!m) return set_err(MG_EINVAL, "mg_relaxation_substeps: null argument");
    if (!(dt_fine > 0.0) || !(dt_e > 0.0) || !(alpha > 0.0) || !std::isfinite(dt_fine) || !std::isfinite(alpha))
        return set_err(MG_EINVAL, "mg_relaxation_substeps: dt_fine, dt_e and alpha must be > 0");
    const double q = alpha * dt_e / dt_fine;  // dt_e may be infinite (no current): one coarse step of the cap
    *m = q >= 1e9 ? 1000000000 : (q < 1.0 ? 1 : (int)std::floor(q));
    return MG_OK;
}

int mg_residual(mg_ctx *c, const double *f_dev, const double *x_dev, double *r_dev, double *rnorm,
                double *bnorm) {
    if (!c || !f_dev || !x_dev) return set_err(MG_EINVAL, "mg_residual: null argument");
    if (!c->coeffs) return set_err(MG_EINVAL, "mg_residual: mg_set_coeffs has not succeeded");
    hipStream_t s = c->stream;
    const Geo G0 = level_geo(c, 0, true);
    const Coef C0 = level_coef(c, 0, false);
    if (r_dev) CK(resid_out(s, G0, C0, x_dev, f_dev, r_dev));
    CK(norm2_resid(s, ST_F64, G0, C0, x_dev, f_dev, c->ws, 0, 1));
    int rc = read_results(c, 2);
    if (rc) return rc;
    if (rnorm) *rnorm = std::sqrt(c->h_pin[0]);
    if (bnorm) *bnorm = std::sqrt(c->h_pin[1]);
    return MG_OK;
}

int mg_smooth(mg_ctx *c, const double *f_dev, double *x_dev, int sweeps) {
    if (!c || !f_dev || !x_dev) return set_err(MG_EINVAL, "mg_smooth: null argument");
    if (!c->coeffs) return set_err(MG_EINVAL, "mg_smooth: mg_set_coeffs has not succeeded");
    if (sweeps < 0) return set_err(MG_EINVAL, "mg_smooth: sweeps must be >= 0");
    hipStream_t s = c->stream;
    const Geo G0 = level_geo(c, 0, true);
    const Coef C0 = level_coef(c, 0, false);
    int zc;
    const int tile = tile_for(c, G0, ST_F64, C0.mode, 0, &zc);
    double *u = x_dev, *t = c->xalt;
    for (int q = 0; q < sweeps; ++q) {
        CK(smooth(s, ST_F64, G0, C0, u, t, f_dev, false, tile, zc));
        std::swap(u, t);
    }
    if (u != x_dev) CK(copy_f64(s, u, x_dev, c->L[0].n));
    CK(hipStreamSynchronize(s));
    return MG_OK;
}

int mg_smooth_level(mg_ctx *c, int l, int store, const double *b_dev, double *x_dev, int sweeps, int tile,
                    int zchunk) {
    if (!c || !b_dev || !x_dev) return set_err(MG_EINVAL, "mg_smooth_level: null argument");
    if (!c->coeffs) return set_err(MG_EINVAL, "mg_smooth_level: mg_set_coeffs has not succeeded");
    if (l < 0 || l >= c->nlev) return set_err(MG_EINVAL, "mg_smooth_level: level %d out of range", l);
    if (store < MG_STORE_F64 || store > MG_STORE_BF16)
        return set_err(MG_EINVAL, "mg_smooth_level: unknown storage type %d", store);
    if (sweeps < 0 || tile < 0 || tile > MG_NUM_TILES || zchunk < 0)
        return set_err(MG_EINVAL, "mg_smooth_level: bad sweeps, tile or zchunk");
    const bool lowp = store != MG_STORE_F64;
    const int st = store == MG_STORE_F64 ? ST_F64 : (store == MG_STORE_F32 ? ST_F32 : ST_BF16);
    if (lowp && st != c->lp_store)
        return set_err(MG_EINVAL, "mg_smooth_level: storage type %d needs a context of that refinement precision",
                       store);
    if (lowp && c->has_eps && l >= 1 && l >= c->tail)
        return set_err(MG_EINVAL, "mg_smooth_level: level %d has no FP32 face coefficients (bottom levels)", l);
    hipStream_t s = c->stream;
    Level &L = c->L[l];
    const size_t n = L.n;
    // the finest FP64 equation carries the boundary values; every other
    // (level, storage) pair is the homogeneous equation the cycles solve
    const bool with_g = l == 0 && !lowp;
    const Geo G = level_geo(c, l, with_g, lowp);
    const Coef C = level_coef(c, l, lowp);
    // coefficients stored multiplied by cscale (every coarse FP64 face of a
    // mixed-precision context, every FP32 copy): scale the right-hand side alike
    const double fac = (lowp || l >= 1) ? c->cscale : 1.0;
    int zc;
    int t = tile_for(c, G, st, C.mode, l, &zc);
    if (tile > 0) t = tile;
    if (zchunk > 0) zc = zchunk;
    else if (tile > 0) zc = default_zchunk(G, t, st, C.mode);
    void *u, *w;
    const void *b;
    if (!lowp && l == 0) {
        u = x_dev;
        w = c->xalt;
        if (fac != 1.0) return set_err(MG_EINVAL, "mg_smooth_level: internal scale mismatch");
        b = b_dev;
    } else {
        u = lowp ? L.ul : (void *)L.u;
        w = lowp ? L.tl : (void *)L.t;
        void *bw = lowp ? L.bl : (void *)L.b;
        CK(convert(s, x_dev, st, u, n, 1.0));
        CK(convert(s, b_dev, st, bw, n, fac));
        b = bw;
    }
    for (int q = 0; q < sweeps; ++q) {
        CK(smooth(s, st, G, C, u, w, b, false, t, zc));
        std::swap(u, w);
    }
    if (u != x_dev) CK(convert_back(s, u, st, x_dev, n, 1.0));
    CK(hipStreamSynchronize(s));
    return MG_OK;
}

int mg_set_option(mg_ctx *c, int key, double value) {
    if (!c) return set_err(MG_EINVAL, "mg_set_option: null context");
    switch (key) {
        case MG_OPT_CORRECTION_WEIGHT:
            if (!(value > 0.0 && value <= 4.0))
                return set_err(MG_EINVAL, "mg_set_option: the correction weight must be in (0, 4]");
            c->corr_w = value;
            c->version++;  // a cached batch plan holds the old weight
            return MG_OK;
    }
    return set_err(MG_EINVAL, "mg_set_option: unknown option %d", key);
}

int mg_prolong_add(mg_ctx *c, int l, const double *e_dev, double *u_dev) {
    if (!c || !e_dev || !u_dev) return set_err(MG_EINVAL, "mg_prolong_add: null argument");
    if (l < 0 || l >= c->nlev - 1) return set_err(MG_EINVAL, "mg_prolong_add: level %d has no coarser level", l);
    hipStream_t s = c->stream;
    const Geo G = level_geo(c, l, false), Gc = level_geo(c, l + 1, false);
    CK(prolong_add(s, ST_F64, G, u_dev, ST_F64, Gc, e_dev, nullptr));
    CK(hipStreamSynchronize(s));
    return MG_OK;
}

int mg_num_levels(const mg_ctx *c) { return c ? c->nlev : 0; }

int mg_level_dims(const mg_ctx *c, int l, int *nx, int *ny, int *nz) {
    if (!c || l < 0 || l >= c->nlev) return set_err(MG_EINVAL, "mg_level_dims: bad level");
    if (nx) *nx = c->L[l].nx;
    if (ny) *ny = c->L[l].ny;
    if (nz) *nz = c->L[l].nz;
    return MG_OK;
}

int mg_tile_shape(int t, int *tx, int *ty) {
    if (t < 1 || t > MG_NUM_TILES) return set_err(MG_EINVAL, "mg_tile_shape: tile must be 1..%d", MG_NUM_TILES);
    tile_shape(t, tx, ty);
    return MG_OK;
}

int mg_set_tiling(mg_ctx *c, int tile, int zchunk) {
    if (!c) return set_err(MG_EINVAL, "mg_set_tiling: null context");
    if (tile < 0 || tile > MG_NUM_TILES || zchunk < 0)
        return set_err(MG_EINVAL, "mg_set_tiling: tile must be 0..%d and zchunk >= 0", MG_NUM_TILES);
    c->tile64 = c->tile_lp = tile;
    c->zc64 = c->zc_lp = zchunk;
    return MG_OK;
}

int mg_timing(mg_ctx *c, int enable) {
    if (!c) return set_err(MG_EINVAL, "mg_timing: null context");
    if (enable && c->ev.empty()) {
        c->ev.resize(1024);
        // the events only bracket kernels for their timestamps: they need no
        // system-scope release, which made each pair read about 2 us longer
        // than the kernel it brackets
        for (auto &e : c->ev) CK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
        c->ev_bytes.resize(512);
        c->ev_step.resize(512);
    }
    c->timing = enable != 0;
    c->ev_used = 0;
    c->t_launches = 0;
    c->t_ms = 0.0;
    c->t_bytes = 0.0;
    c->t_kernel.clear();
    return MG_OK;
}

int mg_timing_read(const mg_ctx *c, long *launches, double *ms, double *bytes, const char **kernel) {
    if (!c) return set_err(MG_EINVAL, "mg_timing_read: null context");
    if (launches) *launches = c->t_launches;
    if (ms) *ms = c->t_ms;
    if (bytes) *bytes = c->t_bytes;
    if (kernel) *kernel = c->t_kernel.c_str();
    return MG_OK;
}

}  // extern "C"
