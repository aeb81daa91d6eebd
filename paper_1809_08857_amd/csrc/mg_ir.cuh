// FP64 refinement pass of the mixed-precision solves, shared by the single
// and the batched engine.
#pragma once

#include "mg_stencil.cuh"

namespace mg {

// xn = x + e * se_inv (FP64 + low precision), r = b - A xn in FP64, r * sc
// stored in the low-precision type, ||r||^2 (and with bslot >= 0 also
// ||b + boundary terms||^2) added to sr (sb).  zero_x: x is taken as 0
// (nothing is read) and xout receives zeros.  se and sc are the powers of two
// of the residual scaling (cast_scale): se undoes the scale of the
// right-hand side that produced e, sc keeps the stored residual within the
// range of the storage type.
//
// One call covers one tile: a TX x TY tile of columns (one thread each)
// marching up a chunk of z planes.  xn (and eps) of planes k-1, k, k+1 stay
// in the thread's registers; the in-plane neighbours of plane k come from an
// LDS plane with a one-cell halo (two buffers by plane parity, so one
// barrier per plane).  Edge threads also carry the halo cell beyond their
// edge; neighbours outside the box are never read.  A workgroup that covers
// several tiles separates them by a barrier (ir_tiles).
//
// The raw loads of a step (own column plane k+3, halo cells and b of plane
// k+2) go to one of two register sets, alternating by step (the loop is
// unrolled by two, so the sets are fixed registers): a value is consumed at
// the end of the step after the one that loaded it, and no load is waited
// for in the step that issues it.
template <class TL, int MODE, bool HAS_E, int TX, int TY>
__device__ __forceinline__ void ir_col_body(const double *__restrict__ x, const TL *__restrict__ e,
                                            double *__restrict__ xout, const double *__restrict__ b,
                                            const double *__restrict__ eps, const Geo &G, TL *__restrict__ rl,
                                            int bslot, int cz, int tiles_x, int tiles_y, int blk, bool zero_x,
                                            double se_inv, double sc, double &sr, double &sb) {
    constexpr bool CELL = (MODE == COEF_CELL);
    __shared__ double su[2][TY + 2][TX + 2];
    __shared__ double se[CELL ? 2 : 1][CELL ? TY + 2 : 1][CELL ? TX + 2 : 1];
    const int tx = blk % tiles_x, rest = blk / tiles_x;
    const int ty = rest % tiles_y, tc = rest / tiles_y;
    const int x0 = tx * TX, y0 = ty * TY, z0 = tc * cz;
    const int nx = G.nx, ny = G.ny, nz = G.nz;
    const int z1 = min(z0 + cz, nz);
    const size_t plane = (size_t)nx * ny;
    const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
    const int i = x0 + lx, j = y0 + ly;
    const bool inc = i < nx && j < ny;
    const size_t col = inc ? (size_t)j * nx + i : 0;
    // halo roles: x-edge threads carry (i -/+ 1, j), y-edge threads (i, j -/+ 1)
    const int hxi = lx == 0 ? i - 1 : (lx == TX - 1 ? i + 1 : -1);
    const int hyj = ly == 0 ? j - 1 : (ly == TY - 1 ? j + 1 : -1);
    const bool hx = hxi >= 0 && hxi < nx && j < ny;
    const bool hy = hyj >= 0 && hyj < ny && i < nx;
    const size_t colx = hx ? (size_t)j * nx + hxi : 0;
    const size_t coly = hy ? (size_t)hyj * nx + i : 0;
    const int sxl = lx == 0 ? 0 : TX + 1, syl = ly == 0 ? 0 : TY + 1;

    // Loads go to a clamped address (a plane outside the box reads the
    // nearest one, a cell outside the box its column's first cell) and are
    // masked where the value is consumed, one step later: a load under a
    // branch would be waited for inside the branch.
    auto at = [&](size_t c, int k) { return (size_t)min(max(k, 0), nz - 1) * plane + c; };
    struct XR { double x; double e; };  // raw x and e of one cell
    auto ldx = [&](size_t c, int k) -> XR {
        XR r{0.0, 0.0};
        if (!zero_x) {  // uniform
            r.x = x[at(c, k)];
            if constexpr (HAS_E) r.e = (double)Num<TL>::ld(e[at(c, k)]) * se_inv;
        }
        return r;
    };
    auto xval = [&](bool ok, int k, const XR &r) -> double {
        return (ok && k >= 0 && k < nz) ? r.x + r.e : 0.0;
    };
    auto lde = [&](size_t c, int k) -> double {
        if constexpr (CELL) return eps[at(c, k)];
        else return 1.0;
    };
    auto eval = [&](bool ok, int k, double v) -> double { return (ok && k >= 0 && k < nz) ? v : 1.0; };
    // own column: planes k-1, k, k+1 and the prefetch k+2; halo: k and k+1
    double um = xval(inc, z0 - 1, ldx(col, z0 - 1)), u0 = xval(inc, z0, ldx(col, z0));
    double up = xval(inc, z0 + 1, ldx(col, z0 + 1));
    double em = eval(inc, z0 - 1, lde(col, z0 - 1)), e0 = eval(inc, z0, lde(col, z0));
    double ep = eval(inc, z0 + 1, lde(col, z0 + 1));
    double hx0 = xval(hx, z0, ldx(colx, z0)), hy0 = xval(hy, z0, ldx(coly, z0));
    double ehx0 = eval(hx, z0, lde(colx, z0)), ehy0 = eval(hy, z0, lde(coly, z0));
    double b0 = b[at(col, z0)];
    // raw loads of one step: own column (x, e, eps), halo cells, b
    struct Raw { XR u, hx, hy; double e, ehx, ehy, b; };
    auto issue = [&](Raw &r, int k) {  // own plane k + 1, halo and b of plane k
        r.u = ldx(col, k + 1), r.hx = ldx(colx, k), r.hy = ldx(coly, k);
        r.e = lde(col, k + 1), r.ehx = lde(colx, k), r.ehy = lde(coly, k);
        r.b = b[at(col, k)];
    };
    Raw ra, rb;
    issue(rb, z0 + 1);  // consumed at the end of step z0
    // step k: issue own plane k+3 and halo/b of plane k+2 into L, compute
    // plane k, then move in own plane k+2 and halo/b of plane k+1 from C
    auto step = [&](int k, Raw &L, const Raw &C) __attribute__((always_inline)) {
        issue(L, k + 2);
        // publish plane k
        const int q = k & 1;
        su[q][ly + 1][lx + 1] = u0;
        if (lx == 0 || lx == TX - 1) su[q][ly + 1][sxl] = hx0;
        if (ly == 0 || ly == TY - 1) su[q][syl][lx + 1] = hy0;
        if constexpr (CELL) {
            se[q][ly + 1][lx + 1] = e0;
            if (lx == 0 || lx == TX - 1) se[q][ly + 1][sxl] = ehx0;
            if (ly == 0 || ly == TY - 1) se[q][syl][lx + 1] = ehy0;
        }
        lds_barrier();
        if (inc) {
            auto un = [&](int d) -> double {
                switch (d) {
                    case 0: return su[q][ly + 1][lx];
                    case 1: return su[q][ly + 1][lx + 2];
                    case 2: return su[q][ly][lx + 1];
                    case 3: return su[q][ly + 2][lx + 1];
                    case 4: return um;
                    default: return up;
                }
            };
            auto en = [&](int d) -> double {
                if constexpr (CELL) {
                    switch (d) {
                        case 0: return se[q][ly + 1][lx];
                        case 1: return se[q][ly + 1][lx + 2];
                        case 2: return se[q][ly][lx + 1];
                        case 3: return se[q][ly + 2][lx + 1];
                        case 4: return em;
                        default: return ep;
                    }
                } else {
                    return 1.0;
                }
            };
            double off, dg;
            six_faces<double, MODE>(G, i, j, k, CELL ? e0 : 1.0, un, en, [&](int) { return 1.0; }, off, dg);
            const size_t p = (size_t)k * plane + col;
            if (HAS_E || zero_x) xout[p] = u0;
            const double r = b0 - G.a * u0 - G.ih2 * (dg * u0 - off);
            rl[p] = Num<TL>::cv(typename Num<TL>::C(r * sc));
            sr += r * r;
            if (bslot >= 0) {  // b plus the boundary terms of the Dirichlet faces the cell touches
                const bool at[6] = {i == 0, i == nx - 1, j == 0, j == ny - 1, k == 0, k == nz - 1};
                double add = 0.0;
#pragma unroll
                for (int d = 0; d < 6; ++d)
                    if (at[d] && ((G.bcmask >> d) & 1)) add += 2.0 * (CELL ? e0 : 1.0) * G.g[d];
                const double bb = b0 + G.ih2 * add;
                sb += bb * bb;
            }
        }
        um = u0, u0 = up, up = xval(inc, k + 2, C.u);
        em = e0, e0 = ep, ep = eval(inc, k + 2, C.e);
        hx0 = xval(hx, k + 1, C.hx), hy0 = xval(hy, k + 1, C.hy);
        ehx0 = eval(hx, k + 1, C.ehx), ehy0 = eval(hy, k + 1, C.ehy);
        b0 = C.b;
    };
    for (int k = z0; k < z1; k += 2) {
        step(k, ra, rb);
        if (k + 1 >= z1) break;
        step(k + 1, rb, ra);
    }
}

// The tiles [first, nblk) with stride `stride` of one refinement pass, run
// by one workgroup, whose partial sums it stores in ws slot `slot` at
// position `wg`; REMAP: tile t is tile xcd_remap(t, nblk) of the grid.  The
// scales: the residual is stored times sc, where sc0 > 0 is the cast scale
// of this pass (its first pass), else it is read from scl[0].  The inner
// cycle solves (cs A) e' = sc r with its coefficients multiplied by cs, so
// the correction is e = e' * cs / scl[1] (scl[1]: the sc of the pass that
// produced e's right-hand side).
template <class TL, int MODE, bool HAS_E, int TX, int TY, bool REMAP>
__device__ __forceinline__ void ir_tiles(const double *__restrict__ x, const TL *__restrict__ e,
                                         double *__restrict__ xout, const double *__restrict__ b,
                                         const double *__restrict__ eps, const Geo &G, TL *__restrict__ rl,
                                         const RedWs &ws, int slot, int bslot, int cz, int tiles_x, int tiles_y,
                                         int first, int nblk, int stride, int wg, bool zero_x,
                                         const double *__restrict__ scl, double sc0, double cs) {
    const double sc = sc0 > 0.0 ? sc0 : scl[0];
    const double se_inv = HAS_E ? cs / scl[1] : 1.0;  // powers of two: exact
    double sr = 0.0, sb = 0.0;
    for (int t = first; t < nblk; t += stride) {
        if (t != first) lds_barrier();  // the previous tile's last plane is still being read
        ir_col_body<TL, MODE, HAS_E, TX, TY>(x, e, xout, b, eps, G, rl, bslot, cz, tiles_x, tiles_y,
                                             REMAP ? xcd_remap(t, nblk) : t, zero_x, se_inv, sc, sr, sb);
    }
    reduce2_finish<TX * TY>(sr, sb, ws, slot, wg);
}

// Final sum of a refinement pass (one workgroup): the norms and the
// convergence flag as reduce2_final_body, then the scales of the next pass.
__device__ __forceinline__ void ir_final_body(const RedWs &ws, int slot, int bslot, int nb, int ref_slot,
                                              double rtol2, int *done, double *scl, double sc0, double n) {
    reduce2_final_body(ws, slot, bslot, nb, ref_slot, rtol2, done);
    if (threadIdx.x == 0) {
        scl[1] = sc0 > 0.0 ? sc0 : scl[0];
        scl[0] = cast_scale(ws.result[slot], n);
    }
}

}  // namespace mg
