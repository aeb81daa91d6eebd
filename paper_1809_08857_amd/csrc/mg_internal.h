// Internal declarations of the multigrid engine (kernels <-> host driver).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cmath>
#include <cstddef>
#include <cstdint>

namespace mg {

using bf16 = __hip_bfloat16;

// Storage type of a field or coefficient array.
enum Store { ST_F64 = 0, ST_F32 = 1, ST_BF16 = 2 };

// How the face coefficient beta_f of the operator is obtained.
//   CONST: beta = 1 everywhere (photon groups).
//   CELL : harmonic mean of the cell coefficient, computed in the kernel.
//   FACE : stored face arrays (coarse levels: mean of the 4 fine faces).
// COEF_FACED: stored faces plus a per-cell extra diagonal (FP64 only).
enum CoefMode { COEF_CONST = 0, COEF_CELL = 1, COEF_FACE = 2, COEF_FACED = 3 };
constexpr bool is_face_mode(int m) { return m == COEF_FACE || m == COEF_FACED; }

inline size_t store_size(int st) { return st == ST_F64 ? 8 : (st == ST_F32 ? 4 : 2); }

// Geometry and scalar data of one level's operator.
struct Geo {
    int nx, ny, nz;
    int bcmask;     // bit f set: face f (x-,x+,y-,y+,z-,z+) is Dirichlet
    double h2;      // h^2
    double ah2;     // a h^2
    double ih2;     // 1 / h^2
    double a;
    double g[6];    // Dirichlet values (0 for correction equations)
    double cw;      // weight of the coarse correction prolongated into this level (1 by default)
};

// Coefficient arrays of one level, in the level's storage type.
struct Coef {
    int mode;           // CoefMode
    const void *eps;    // CELL: nx*ny*nz
    const void *bx;     // FACE: (nx+1)*ny*nz
    const void *by;     // FACE: nx*(ny+1)*nz
    const void *bz;     // FACE: nx*ny*(nz+1)
    const double *dd;   // FACED: nx*ny*nz, added to a cell by cell
};

// Deterministic reduction workspace: per-block partial sums (kMaxRedBlocks
// pairs per slot) and the result slots.
struct RedWs {
    double *partials;
    double *result;
};
constexpr int kMaxRedBlocks = 2048;
// Largest accepted cell coefficient (the smoothers encode Dirichlet box
// faces with a coefficient of 2^400 that must dominate every cell's).
constexpr double kMaxCellCoef = 1e100;
// Largest x-y plane (cells): the stencil kernels address a plane with
// 32-bit byte offsets from a per-plane base.
constexpr long kMaxPlaneCells = 1L << 28;
constexpr int kRedSlots = 8;
// Result slots of the refinement pass's residual scales (powers of two):
// [kSlotScale] the scale applied to the residual before its cast to the
// inner storage type, [kSlotScale + 1] the scale of the rhs that produced
// the correction being added (see ir_update_resid).
constexpr int kSlotScale = 4;

// Power-of-two scale for the low-precision copy of a residual whose sum of
// squares over n cells is ss: 1 while the root-mean-square value lies in
// [2^-40, 2^40] (FP32 and BF16 hold such values and the inner cycle's
// intermediate sums with ample range), else 2^-e with e the binary exponent
// of the root mean square, which brings it into [1/2, 1).  A power of two
// leaves every rounding of the inner cycle unchanged.
__host__ __device__ inline double cast_scale_rms(double rms) {
    if (!(rms > 0.0) || !(rms < 1e300)) return 1.0;
    int e;
    (void)frexp(rms, &e);
    if (e >= -40 && e <= 40) return 1.0;
    return ldexp(1.0, -e);
}
__host__ __device__ inline double cast_scale(double ss, double n) { return cast_scale_rms(sqrt(ss / n)); }

// Fused convergence test of a residual pass: reduce ||r||^2 into
// ws.result[slot] (slot < 0: no norm), and set *done_out when it is
// <= rtol2 * ws.result[ref_slot].  Kernels given done_in return at once
// when *done_in is set (the solve has converged).
struct RrCheck {
    RedWs ws{};
    int slot = -1;
    int ref_slot = -1;
    double rtol2 = 0.0;
    int *done_out = nullptr;
    const int *done_in = nullptr;
};

// ------------------------------------------------------------ launchers

// Brick launch shape: BX x BY threads (BX*BY = 256) over nxi items along x
// and ny rows; blockIdx.z runs over nz planes in chunks of *kz so that at
// most max_blocks blocks are launched (0 = one plane per block).
inline void brick_shape(int nxi, int ny, int nz, int max_blocks, dim3 *grid, dim3 *block, int *kz) {
    int bx = nxi >= 64 ? 64 : (nxi >= 32 ? 32 : 16);
    int by = 256 / bx;
    const int gx = (nxi + bx - 1) / bx, gy = (ny + by - 1) / by;
    int gz = nz, z = 1;
    if (max_blocks > 0) {
        long room = max_blocks / ((long)gx * gy);
        if (room < 1) room = 1;
        if (gz > room) gz = (int)room;
        z = (nz + gz - 1) / gz;
        gz = (nz + z - 1) / z;
    }
    *grid = dim3(gx, gy, gz);
    *block = dim3(bx, by, 1);
    *kz = z;
}


// All launchers enqueue on `s` and return hipGetLastError().

// Tile variants of the fused red-black smoother: (TX, TY) per index 1..6.
constexpr int kNumTiles = 6;
void tile_shape(int t, int *tx, int *ty);
int default_tile(const Geo &G, int st, int mode);
int default_zchunk(const Geo &G, int tile, int st, int mode);

// One fused red-black Gauss-Seidel sweep, out of place: uout = sweep(uin).
// zero_in: treat uin as identically zero (uin is not read).
hipError_t smooth(hipStream_t s, int st, const Geo &G, const Coef &C, const void *uin, void *uout,
                  const void *b, bool zero_in, int tile, int zchunk, const int *done = nullptr);

// Residual of level (G,C) restricted to the coarse right-hand side:
// bc[I] = mean over the 8 children of (b - A u).  Fine store `st`,
// coarse store `stc`.
hipError_t resid_restrict(hipStream_t s, int st, const Geo &G, const Coef &C, const void *u,
                          const void *b, int stc, void *bc, const RrCheck &chk);

// u += P e (cell-centred trilinear, ghost -e / +e at Dirichlet / Neumann
// faces).  e has the coarse geometry Gc and store stc.
hipError_t prolong_add(hipStream_t s, int st, const Geo &G, void *u, int stc, const Geo &Gc,
                       const void *e, const int *done = nullptr);

// ||b - A u||^2 (slot) and, if bslot >= 0, ||b||^2 including boundary
// terms (bslot), FP64 accumulation, deterministic.
hipError_t norm2_resid(hipStream_t s, int st, const Geo &G, const Coef &C, const void *u,
                       const void *b, const RedWs &ws, int slot, int bslot,
                       const RrCheck *chk = nullptr);

// y = alpha x + beta A x with zero boundary values (FP64).
hipError_t apply_op(hipStream_t s, const Geo &G, const Coef &C, double alpha, double beta, const double *x,
                    double *y);

// E = -grad(phi) at the cell centres (central differences over two cells,
// ghost values 2g - phi beyond Dirichlet faces and phi beyond Neumann
// faces); any of ex, ey, ez may be null (not written).  ws.result[slot] =
// max |E| and ws.result[slot + 1] = max sigma |E| (0 without sigma).
hipError_t field(hipStream_t s, const Geo &G, double h, const double *phi, const double *sigma, double *ex,
                 double *ey, double *ez, const RedWs &ws, int slot);

// Residual in FP64 written out: r = b - A u (all FP64).
hipError_t resid_out(hipStream_t s, const Geo &G, const Coef &C, const double *u, const double *b,
                     double *r);

// Mixed precision: r_lp = b - A x (FP64 arithmetic) cast to `stl`,
// plus ||r||^2 into `slot`.  If e != nullptr the correction is applied
// first: xout = x + e (e in store stl), and the residual is that of xout.
// Final sum of the partials a reducing kernel stored in slot `slot` (nb
// workgroups): result[slot] (and result[bslot] for the second sum) and the
// convergence flag (skipped when done_in is set).
hipError_t reduce2_final(hipStream_t s, const RedWs &ws, int slot, int bslot, int nb, int ref_slot, double rtol2,
                         int *done, const int *done_in);
//
// Scales (see cast_scale): the residual is stored as r * sc, where sc = sc0
// if sc0 > 0, else ws.result[kSlotScale]; the inner cycle solves
// (cs A) e' = sc r with its coefficients multiplied by the power of two cs,
// so e is added as e * cs / ws.result[kSlotScale + 1].  The final sum then
// moves the scale used into slot kSlotScale + 1 and stores
// cast_scale(||r||^2, n) in slot kSlotScale for the next pass.
hipError_t ir_update_resid(hipStream_t s, const Geo &G, const Coef &C, const double *x,
                           const void *e, double *xout, const double *b, int stl, void *r_lp,
                           const RrCheck &chk, double sc0, double cs);
// p[0..n) *= factor (FP64).
hipError_t scale_f64(hipStream_t s, double *p, size_t n, double factor);
// max and min of x[0..n) into ws.result[slot] and ws.result[slot + 1].
hipError_t minmax(hipStream_t s, const double *x, size_t n, const RedWs &ws, int slot);

// Setup kernels.
hipError_t faces_from_cell(hipStream_t s, const Geo &G, const double *eps, double *bx, double *by,
                           double *bz);
hipError_t coarsen_faces(hipStream_t s, const Geo &Gf, const double *fbx, const double *fby,
                         const double *fbz, const Geo &Gc, double *cbx, double *cby, double *cbz);
// dst = src * factor rounded to the storage type st (round to nearest even).
hipError_t convert(hipStream_t s, const double *src, int st, void *dst, size_t n, double factor = 1.0);
// src (storage type st) to FP64: dst = src * factor.
hipError_t convert_back(hipStream_t s, const void *src, int st, double *dst, size_t n, double factor = 1.0);
// count of entries that are not finite or not > 0, into ws slot (as double)
hipError_t count_bad(hipStream_t s, const double *x, size_t n, const RedWs &ws, int slot);
hipError_t count_outside(hipStream_t s, const double *x, size_t n, double lo, double hi, const RedWs &ws,
                         int slot);
hipError_t count_singular(hipStream_t s, const Geo &G, const double *bx, const double *by, const double *bz,
                          const double *d, const RedWs &ws, int slot);
hipError_t coarsen_cells(hipStream_t s, const Geo &Gf, const double *f, const Geo &Gc, double *c);
hipError_t fill_zero(hipStream_t s, void *p, size_t bytes, const int *done = nullptr);
hipError_t copy_f64(hipStream_t s, const double *src, double *dst, size_t n, const int *done = nullptr);

// ------------------------------------------------------------ bottom
constexpr int kTailMaxLevels = 12;
constexpr int kTailLdsDoubles = 16384;  // 128 KiB of LDS

struct TailLevel {
    int nx, ny, nz;
    double h2, ah2;
    const double *bx, *by, *bz;  // FACE arrays (FP64) or null (CONST)
    const double *dd;            // FACED: per-cell extra diagonal (read from memory)
    int off_u, off_b;            // LDS offsets (doubles) of iterate and right-hand side
    int off_fx, off_fy, off_fz;  // LDS offsets of the staged face coefficients (FACE)
};

struct TailDesc {
    int nlev;             // levels handled, >= 1 (the last is the coarsest)
    int mode;             // COEF_CONST, COEF_FACE or COEF_FACED
    int bcmask;
    double g[6];          // Dirichlet values of the top level (0 for corrections)
    int nu1, nu2, ncyc;   // smoothing sweeps and V-cycles inside the bottom
    int off_p, off_q;     // LDS offsets of the CG vectors of the coarsest
    int cg_maxit;
    double cg_rtol;
    int stage;            // 1: FACE coefficients staged in LDS, 0: read from memory
    TailLevel L[kTailMaxLevels];
};

// Solve the top tail level: u_out = (approximate) A^-1 b_in, b_in/u_out in
// store st.  If u_in != nullptr it is the starting iterate (else zero).
hipError_t tail_solve(hipStream_t s, int st, const TailDesc &D, const void *b_in, const void *u_in,
                      void *u_out, const int *done = nullptr);
bool tail_layout(TailDesc &D);  // assigns LDS offsets; false if it does not fit

// Arrays of one problem of a batched bottom solve (zero start).
struct TailIo {
    const void *b;
    void *u;
    const int *done;
};
hipError_t tail_solve_batched(hipStream_t s, int st, const TailDesc *descs, const TailIo *io, int count);

}  // namespace mg
