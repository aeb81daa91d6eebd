// Context layout shared by the host-side parts of the engine
// (mg_engine.hip, mg_batched.hip, mg_autotune.hip).
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <string>
#include <vector>

#include "mg.h"
#include "mg_internal.h"

namespace mg {

constexpr int kMaxLevels = 24;

struct Level {
    int nx = 0, ny = 0, nz = 0;
    size_t n = 0;
    double h = 0.0;
    double *fbx = nullptr, *fby = nullptr, *fbz = nullptr;  // FP64 face coefficients
    void *lbx = nullptr, *lby = nullptr, *lbz = nullptr;    // low-precision copies
    double *u = nullptr, *t = nullptr, *b = nullptr;        // FP64 work (levels >= 1)
    void *ul = nullptr, *tl = nullptr, *bl = nullptr;       // low-precision work
    double *dd = nullptr;                                   // extra diagonal (mg_set_face_coeffs_diag)
};

// One level as seen by a V-cycle: storage type, operator and arrays.
struct LvView {
    int st = ST_F64;
    Geo G{};
    Coef C{};
    size_t n = 0;
    void *u = nullptr, *t = nullptr;
    const void *b = nullptr;
    void *bw = nullptr;      // writable alias of b (target of the restriction)
    bool fixed_u = false;    // u is the caller's array: the result must end there
    bool with_g = false;     // boundary values apply (finest level of the FP64 solve)
};

struct BatchPlan;  // mg_batched.hip

// Divergence test of a sequence of relative residuals (one per cycle): a
// non-finite value, growth by 1e6 over the start, or growth in each of
// kGrowCycles consecutive cycles to more than 10x the smallest value seen.
// A solve stalled at its rounding floor moves by small factors either way
// and is reported as not converged instead.
struct DivergenceWatch {
    static constexpr int kGrowCycles = 4;
    double rmin = HUGE_VAL, last = HUGE_VAL;
    int grow = 0;
    bool diverged(double rel, double rel0) {
        if (!std::isfinite(rel)) return true;
        grow = rel > last ? grow + 1 : 0;
        last = rel;
        rmin = std::min(rmin, rel);
        return rel > 1e6 * std::max(1.0, rel0) || (grow >= kGrowCycles && rel > 10.0 * rmin);
    }
};

}  // namespace mg

struct mg_ctx {
    mg_desc d{};
    hipStream_t stream = nullptr;
    int lp_store = -1;  // ST_F32 / ST_BF16 for refinement, -1 for MG_FP64
    int nlev = 0, tail = 0, tail0 = 0;  // tail: first level of the bottom solver
    mg::Level L[mg::kMaxLevels];
    bool has_eps = false;   // variable coefficients: stored faces on the coarse levels
    bool face0 = false;     // the finest level's faces were given (mg_set_face_coeffs)
    bool has_diag = false;  // faces plus a per-cell diagonal (mg_set_face_coeffs_diag)
    double *eps = nullptr;
    void *eps_lp = nullptr;
    double a = 0.0;
    double cscale = 1.0;  // power of two multiplying the inner (FP32/BF16) operator's coefficients
    double corr_w = 1.0;  // weight of the coarse correction at the finest level (MG_OPT_CORRECTION_WEIGHT)
    int bcmask = 0;
    double g[6] = {0, 0, 0, 0, 0, 0};
    bool coeffs = false;
    unsigned version = 0;  // bumped by every mg_set_coeffs
    unsigned long uid = 0;  // unique per context in the process
    double *xalt = nullptr;
    double *work = nullptr;  // right-hand sides of mg_tga_step (allocated at its first call)
    int *d_done = nullptr;             // device convergence flag of the running solve
    hipEvent_t ev_cyc[2] = {nullptr, nullptr};
    mg::RedWs ws{};
    double *h_pin = nullptr;
    int tile64 = 0, zc64 = 0, tile_lp = 0, zc_lp = 0;
    mg::TailDesc tails[2];  // [0]: homogeneous, [1]: with boundary values
    std::vector<void *> allocs;
    mg::BatchPlan *plan = nullptr;  // cached batch plan owned by this context (first of a batch)
    // measurement hook (mg_timing)
    bool timing = false;
    std::vector<hipEvent_t> ev;  // start/stop pairs
    std::vector<double> ev_bytes;
    std::vector<int> ev_step;  // pipeline step of each timed launch (-1: outside a solve)
    int cur_step = -1;         // check(k) = 2k, advance(k) = 2k + 1
    int ev_used = 0;
    long t_launches = 0;
    double t_ms = 0.0, t_bytes = 0.0;
    std::string t_kernel;
};

namespace mg {

using Ctx = ::mg_ctx;

extern thread_local std::string g_err;
int set_err(int code, const char *fmt, ...);
// Geometry of level l; with_g: the Dirichlet values apply (finest level of
// the FP64 problem); lowp: the inner low-precision operator (coefficients
// multiplied by cscale).
Geo level_geo(const Ctx *c, int l, bool with_g, bool lowp = false);
Coef level_coef(const Ctx *c, int l, bool lowp);
// Sets a and rebuilds the bottom-solver descriptors (host only).
void set_screening(Ctx *c, double a);
// Validation shared by the entry points (MG_OK or MG_EINVAL with a message).
int check_grid(const char *who, const mg_desc *d);
int parse_operator(const char *who, double a, const mg_bcs *bc, int *mask);
void build_tail(const Ctx *c, TailDesc &D, bool with_g);
int tile_for(const Ctx *c, const Geo &G, int st, int mode, int l, int *zc);
int vcycle(Ctx *c, std::vector<LvView> &V, int l, bool zero_start, const int *done = nullptr);
void fp64_view(Ctx *c, std::vector<LvView> &V, const double *f, double *x);
void lowp_view(Ctx *c, std::vector<LvView> &V);
int read_results(Ctx *c, int n);
void batch_release(Ctx *c);
// Adds the timed launches to the totals; launches of pipeline steps after
// max_step (enqueued ahead and skipped once the solve converged) are dropped.
int timing_flush(Ctx *c, int max_step = 1 << 30);

// ||b||^2 of the finest-level FP64 problem (b = f + boundary terms) into
// ws.result[slot] (mg_misc.hip); level 0 is CONST or CELL.
hipError_t norm2_b(hipStream_t s, const Geo &G, const Coef &C, const double *f, const RedWs &ws, int slot);
hipError_t timed_smooth(Ctx *c, int l, const LvView &W, bool zin, int tile, int zc, const int *done = nullptr);

}  // namespace mg
