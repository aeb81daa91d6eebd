// Host launchers of the stencil kernels for one storage type T.  Included
// once per storage type (mg_kern_f64.hip, mg_kern_f32.hip, mg_kern_bf16.hip).
#pragma once

#include <type_traits>

#include "mg_stencil.cuh"

namespace mg {

// (TX, TY) of the smoother tile variants.
constexpr int kTileTX[kNumTiles + 1] = {0, 64, 128, 64, 32, 32, 16};
constexpr int kTileTY[kNumTiles + 1] = {0, 16, 8, 8, 8, 4, 8};

template <class T>
inline void coef_ptrs(const Coef &C, const coef_t<T> *&eps, const coef_t<T> *&bx, const coef_t<T> *&by,
                      const coef_t<T> *&bz) {
    eps = static_cast<const coef_t<T> *>(C.eps);
    bx = static_cast<const coef_t<T> *>(C.bx);
    by = static_cast<const coef_t<T> *>(C.by);
    bz = static_cast<const coef_t<T> *>(C.bz);
}

template <class T, int MODE, int TX, int TY>
hipError_t smooth_tile(hipStream_t s, const Geo &G, const Coef &Cf, const void *uin, void *uout,
                       const void *b, bool zero_in, int cz, const int *done) {
    const coef_t<T> *eps, *bx, *by, *bz;
    coef_ptrs<T>(Cf, eps, bx, by, bz);
    const int tiles_x = (G.nx + TX - 1) / TX, tiles_y = (G.ny + TY - 1) / TY;
    const int chunks = (G.nz + cz - 1) / cz;
    const int nblk = tiles_x * tiles_y * chunks;
    const dim3 grid(nblk), block((TX + 4) / 2 * (TY + 4));
    SmoothArgs<T> A{static_cast<const T *>(uin), static_cast<T *>(uout), static_cast<const T *>(b), eps, bx,
                    by, bz, G, cz, tiles_x, tiles_y, nblk, done, Cf.dd};
    constexpr int PD = kSmoothPDOf<T>;
    const bool even = (G.nx & 1) == 0;
    if (zero_in && even)
        hipLaunchKernelGGL((rbgs_col_k<T, MODE, TX, TY, true, PD, true>), grid, block, 0, s, A);
    else if (zero_in)
        hipLaunchKernelGGL((rbgs_col_k<T, MODE, TX, TY, true, PD, false>), grid, block, 0, s, A);
    else if (even)
        hipLaunchKernelGGL((rbgs_col_k<T, MODE, TX, TY, false, PD, true>), grid, block, 0, s, A);
    else
        hipLaunchKernelGGL((rbgs_col_k<T, MODE, TX, TY, false, PD, false>), grid, block, 0, s, A);
    return hipGetLastError();
}

template <class T, int MODE>
hipError_t smooth_mode(hipStream_t s, const Geo &G, const Coef &Cf, const void *uin, void *uout,
                       const void *b, bool zero_in, int tile, int cz, const int *done) {
    switch (tile) {
        case 1: return smooth_tile<T, MODE, 64, 16>(s, G, Cf, uin, uout, b, zero_in, cz, done);
        case 2: return smooth_tile<T, MODE, 128, 8>(s, G, Cf, uin, uout, b, zero_in, cz, done);
        case 3: return smooth_tile<T, MODE, 64, 8>(s, G, Cf, uin, uout, b, zero_in, cz, done);
        case 4: return smooth_tile<T, MODE, 32, 8>(s, G, Cf, uin, uout, b, zero_in, cz, done);
        case 5: return smooth_tile<T, MODE, 32, 4>(s, G, Cf, uin, uout, b, zero_in, cz, done);
        case 6: return smooth_tile<T, MODE, 16, 8>(s, G, Cf, uin, uout, b, zero_in, cz, done);
        default: return hipErrorInvalidValue;
    }
}

template <class T>
hipError_t smooth_T(hipStream_t s, const Geo &G, const Coef &Cf, const void *uin, void *uout,
                    const void *b, bool zero_in, int tile, int cz, const int *done) {
    if (cz < 1) return hipErrorInvalidValue;
    switch (Cf.mode) {
        case COEF_CONST: return smooth_mode<T, COEF_CONST>(s, G, Cf, uin, uout, b, zero_in, tile, cz, done);
        case COEF_CELL: return smooth_mode<T, COEF_CELL>(s, G, Cf, uin, uout, b, zero_in, tile, cz, done);
        case COEF_FACE: return smooth_mode<T, COEF_FACE>(s, G, Cf, uin, uout, b, zero_in, tile, cz, done);
        case COEF_FACED:
            if constexpr (std::is_same<T, double>::value)
                return smooth_mode<T, COEF_FACED>(s, G, Cf, uin, uout, b, zero_in, tile, cz, done);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

template <class T, int MODE, int TX, int TY>
hipError_t rr_tile(hipStream_t s, const Geo &G, const Coef &Cf, const void *u, const void *b, void *bc,
                   const RrCheck &chk) {
    const coef_t<T> *eps, *bx, *by, *bz;
    coef_ptrs<T>(Cf, eps, bx, by, bz);
    const int tiles_x = (G.nx + TX - 1) / TX, tiles_y = (G.ny + TY - 1) / TY;
    const long cols = (long)tiles_x * tiles_y;
    // about as many workgroups as the chip holds at once: two per CU, but one
    // where a 10-wave workgroup of a 64 x 16 tile is all that fits, by its
    // registers per lane: cell permittivity (102-116), stored faces in FP64
    // or FP32 (108-136); beta = 1 (63-86) and BF16 stored faces (96) fit
    // two.  A second round of workgroups measured slower (FP64 cell
    // permittivity at 256^3: 91.6 against 87.3 us)
    constexpr bool kOnePerCu =
        TX * TY >= 1024 && (MODE == COEF_CELL || (MODE != COEF_CONST && !std::is_same<T, bf16>::value));
    constexpr long kTarget = kOnePerCu ? 256 : 512;
    long chunks = (kTarget + cols - 1) / cols;
    long maxch = G.nz / 8;
    if (maxch < 1) maxch = 1;
    if (chunks > maxch) chunks = maxch;
    int cz = (int)((G.nz + chunks - 1) / chunks);
    cz += cz & 1;  // chunks hold whole coarse planes
    const int nblk = tiles_x * tiles_y * ((G.nz + cz - 1) / cz);
    constexpr int NTH = rr_threads<TX, TY>();
    // a checked pass reduces one partial norm per workgroup: at most kMaxRedBlocks
    const int nwg = (chk.slot >= 0 && nblk > kMaxRedBlocks) ? kMaxRedBlocks : nblk;
    RrArgs<T> A{static_cast<const T *>(u), static_cast<const T *>(b), eps, bx, by, bz, G,
                static_cast<T *>(bc), cz, tiles_x, tiles_y, nblk, chk.ws, chk.slot, chk.ref_slot,
                chk.rtol2, chk.done_out, chk.done_in, Cf.dd};
    hipLaunchKernelGGL((rr_col_k<T, MODE, TX, TY, kSmoothPDOf<T>>), dim3(nwg), dim3(NTH), 0, s, A);
    if (hipPeekAtLastError() != hipSuccess) return hipGetLastError();
    if (chk.slot >= 0)
        return reduce2_final(s, chk.ws, chk.slot, -1, nwg, chk.ref_slot, chk.rtol2, chk.done_out, chk.done_in);
    return hipGetLastError();
}

template <class T, int MODE>
hipError_t rr_mode(hipStream_t s, const Geo &G, const Coef &Cf, const void *u, const void *b, void *bc,
                   const RrCheck &chk) {
    if (G.nx >= 64 && G.ny >= 16) return rr_tile<T, MODE, 64, 16>(s, G, Cf, u, b, bc, chk);
    if (G.nx >= 64) return rr_tile<T, MODE, 64, 8>(s, G, Cf, u, b, bc, chk);
    if (G.nx >= 32) return rr_tile<T, MODE, 32, 8>(s, G, Cf, u, b, bc, chk);
    return rr_tile<T, MODE, 16, 8>(s, G, Cf, u, b, bc, chk);
}

template <class T>
hipError_t resid_restrict_T(hipStream_t s, const Geo &G, const Coef &Cf, const void *u,
                            const void *b, void *bc, const RrCheck &chk) {
    if ((G.nx | G.ny | G.nz) & 1) return hipErrorInvalidValue;
    switch (Cf.mode) {
        case COEF_CONST: return rr_mode<T, COEF_CONST>(s, G, Cf, u, b, bc, chk);
        case COEF_CELL: return rr_mode<T, COEF_CELL>(s, G, Cf, u, b, bc, chk);
        case COEF_FACE: return rr_mode<T, COEF_FACE>(s, G, Cf, u, b, bc, chk);
        case COEF_FACED:
            if constexpr (std::is_same<T, double>::value) return rr_mode<T, COEF_FACED>(s, G, Cf, u, b, bc, chk);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

template <class T>
hipError_t prolong_T(hipStream_t s, const Geo &G, void *u, const Geo &Gc, const void *e, const int *done) {
    if ((G.nx | G.ny | G.nz) & 1 || Gc.nx * 2 != G.nx || Gc.ny * 2 != G.ny || Gc.nz * 2 != G.nz)
        return hipErrorInvalidValue;
    constexpr int BX = 64, BY = 4;
    const long cols = (long)((Gc.nx + BX - 1) / BX) * ((G.ny + BY - 1) / BY);
    // about 2048 workgroups, chunks of an even number of fine planes
    long chunks = (2048 + cols - 1) / cols;
    if (chunks > G.nz / 2) chunks = G.nz / 2;
    if (chunks < 1) chunks = 1;
    int kz = (int)((G.nz + chunks - 1) / chunks);
    kz += kz & 1;
    const dim3 grid((Gc.nx + BX - 1) / BX, (G.ny + BY - 1) / BY, (G.nz + kz - 1) / kz), block(BX, BY);
    hipLaunchKernelGGL((prolong_col_k<T, BX, BY>), grid, block, 0, s, static_cast<T *>(u),
                       static_cast<const T *>(e), G, Gc, kz, done);
    return hipGetLastError();
}

template <class T>
hipError_t norm2_T(hipStream_t s, const Geo &G, const Coef &Cf, const void *u, const void *b,
                   const RedWs &ws, int slot, int bslot, const RrCheck *chk) {
    const int ref = chk ? chk->ref_slot : -1;
    const double rt2 = chk ? chk->rtol2 : 0.0;
    int *dout = chk ? chk->done_out : nullptr;
    const int *din = chk ? chk->done_in : nullptr;
    const coef_t<T> *eps, *bx, *by, *bz;
    coef_ptrs<T>(Cf, eps, bx, by, bz);
    dim3 grid, block;
    int kz;
    brick_shape(G.nx, G.ny, G.nz, kMaxRedBlocks, &grid, &block, &kz);
    const int nbrick = (int)(grid.x * grid.y * grid.z);
    const int nwg = nbrick < kMaxRedBlocks ? nbrick : kMaxRedBlocks;
    const T *uu = static_cast<const T *>(u), *bb = static_cast<const T *>(b);
    const int gx = (int)grid.x, gy = (int)grid.y;
    switch (Cf.mode) {
        case COEF_CONST:
            hipLaunchKernelGGL((norm2_resid_k<T, COEF_CONST>), dim3(nwg), block, 0, s, uu, bb, eps,
                               bx, by, bz, G, ws, slot, bslot, kz, gx, gy, nbrick, din, nullptr);
            break;
        case COEF_CELL:
            hipLaunchKernelGGL((norm2_resid_k<T, COEF_CELL>), dim3(nwg), block, 0, s, uu, bb, eps,
                               bx, by, bz, G, ws, slot, bslot, kz, gx, gy, nbrick, din, nullptr);
            break;
        case COEF_FACE:
            hipLaunchKernelGGL((norm2_resid_k<T, COEF_FACE>), dim3(nwg), block, 0, s, uu, bb, eps,
                               bx, by, bz, G, ws, slot, bslot, kz, gx, gy, nbrick, din, nullptr);
            break;
        case COEF_FACED:
            if constexpr (std::is_same<T, double>::value) {
                hipLaunchKernelGGL((norm2_resid_k<T, COEF_FACED>), dim3(nwg), block, 0, s, uu, bb, eps,
                                   bx, by, bz, G, ws, slot, bslot, kz, gx, gy, nbrick, din, Cf.dd);
                break;
            }
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
    if (hipPeekAtLastError() != hipSuccess) return hipGetLastError();
    return reduce2_final(s, ws, slot, bslot, nwg, ref, rt2, dout, din);
}

}  // namespace mg

// Exported per-type entry points (names suffixed by the storage type).
#define MG_DEFINE_TYPE_ENTRIES(T, SUF)                                                              \
    namespace mg {                                                                                  \
    hipError_t smooth_##SUF(hipStream_t s, const Geo &G, const Coef &C, const void *uin, void *uout, \
                            const void *b, bool zin, int tile, int cz, const int *done) {           \
        return smooth_T<T>(s, G, C, uin, uout, b, zin, tile, cz, done);                             \
    }                                                                                               \
    hipError_t resid_restrict_##SUF(hipStream_t s, const Geo &G, const Coef &C, const void *u,       \
                                    const void *b, void *bc, const RrCheck &chk) {                  \
        return resid_restrict_T<T>(s, G, C, u, b, bc, chk);                                         \
    }                                                                                               \
    hipError_t prolong_##SUF(hipStream_t s, const Geo &G, void *u, const Geo &Gc, const void *e,     \
                             const int *done) {                                                     \
        return prolong_T<T>(s, G, u, Gc, e, done);                                                  \
    }                                                                                               \
    hipError_t norm2_##SUF(hipStream_t s, const Geo &G, const Coef &C, const void *u, const void *b, \
                           const RedWs &ws, int slot, int bslot, const RrCheck *chk) {              \
        return norm2_T<T>(s, G, C, u, b, ws, slot, bslot, chk);                                     \
    }                                                                                               \
    }
