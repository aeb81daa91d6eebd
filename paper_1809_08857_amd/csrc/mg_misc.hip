// Set-up kernels, FP64 refinement kernels and the storage-type dispatch of
// the stencil launchers.
#include "mg_ir.cuh"
#include "mg_stencil.cuh"

namespace mg {

#define MG_DECLARE_TYPE_ENTRIES(SUF)                                                                \
    hipError_t smooth_##SUF(hipStream_t, const Geo &, const Coef &, const void *, void *,          \
                            const void *, bool, int, int, const int *);                             \
    hipError_t resid_restrict_##SUF(hipStream_t, const Geo &, const Coef &, const void *,           \
                                    const void *, void *, const RrCheck &);                         \
    hipError_t prolong_##SUF(hipStream_t, const Geo &, void *, const Geo &, const void *,           \
                             const int *);                                                          \
    hipError_t norm2_##SUF(hipStream_t, const Geo &, const Coef &, const void *, const void *,      \
                           const RedWs &, int, int, const RrCheck *);
MG_DECLARE_TYPE_ENTRIES(f64)
MG_DECLARE_TYPE_ENTRIES(f32)
MG_DECLARE_TYPE_ENTRIES(bf16)

hipError_t smooth(hipStream_t s, int st, const Geo &G, const Coef &C, const void *uin, void *uout,
                  const void *b, bool zero_in, int tile, int zchunk, const int *done) {
    switch (st) {
        case ST_F64: return smooth_f64(s, G, C, uin, uout, b, zero_in, tile, zchunk, done);
        case ST_F32: return smooth_f32(s, G, C, uin, uout, b, zero_in, tile, zchunk, done);
        case ST_BF16: return smooth_bf16(s, G, C, uin, uout, b, zero_in, tile, zchunk, done);
    }
    return hipErrorInvalidValue;
}

hipError_t resid_restrict(hipStream_t s, int st, const Geo &G, const Coef &C, const void *u,
                          const void *b, int stc, void *bc, const RrCheck &chk) {
    if (stc != st) return hipErrorInvalidValue;
    switch (st) {
        case ST_F64: return resid_restrict_f64(s, G, C, u, b, bc, chk);
        case ST_F32: return resid_restrict_f32(s, G, C, u, b, bc, chk);
        case ST_BF16: return resid_restrict_bf16(s, G, C, u, b, bc, chk);
    }
    return hipErrorInvalidValue;
}

hipError_t prolong_add(hipStream_t s, int st, const Geo &G, void *u, int stc, const Geo &Gc,
                       const void *e, const int *done) {
    if (stc != st) return hipErrorInvalidValue;
    switch (st) {
        case ST_F64: return prolong_f64(s, G, u, Gc, e, done);
        case ST_F32: return prolong_f32(s, G, u, Gc, e, done);
        case ST_BF16: return prolong_bf16(s, G, u, Gc, e, done);
    }
    return hipErrorInvalidValue;
}

hipError_t norm2_resid(hipStream_t s, int st, const Geo &G, const Coef &C, const void *u,
                       const void *b, const RedWs &ws, int slot, int bslot, const RrCheck *chk) {
    switch (st) {
        case ST_F64: return norm2_f64(s, G, C, u, b, ws, slot, bslot, chk);
        case ST_F32: return norm2_f32(s, G, C, u, b, ws, slot, bslot, chk);
        case ST_BF16: return norm2_bf16(s, G, C, u, b, ws, slot, bslot, chk);
    }
    return hipErrorInvalidValue;
}

// Final sum of a two-launch reduction (see reduce2_finish).
__global__ __launch_bounds__(kFinalThreads) void reduce2_final_k(RedWs ws, int slot, int bslot, int nb,
                                                                 int ref_slot, double rtol2, int *done,
                                                                 const int *done_in) {
    if (done_in && *done_in) return;  // the reducing kernel returned at once as well
    reduce2_final_body(ws, slot, bslot, nb, ref_slot, rtol2, done);
}

hipError_t reduce2_final(hipStream_t s, const RedWs &ws, int slot, int bslot, int nb, int ref_slot, double rtol2,
                         int *done, const int *done_in) {
    if (nb < 1 || nb > kMaxRedBlocks) return hipErrorInvalidValue;
    hipLaunchKernelGGL(reduce2_final_k, dim3(1), dim3(kFinalThreads), 0, s, ws, slot, bslot, nb, ref_slot, rtol2,
                       done, done_in);
    return hipGetLastError();
}

// ||b||^2 with b = f + h^-2 sum_Dirichlet 2 beta g (the relative-residual
// reference, and the residual of a zero iterate): one read of f per cell,
// beta (cell coefficient, or 1) only on boundary cells.  Brick of kz
// planes per block, loads of four planes in flight.
template <int MODE>
__global__ __launch_bounds__(256) void norm2_b_k(const double *__restrict__ f, const double *__restrict__ eps,
                                                 const double *__restrict__ bx, const double *__restrict__ by,
                                                 const double *__restrict__ bz, Geo G, RedWs ws, int slot, int kz,
                                                 int gx, int gy, int nbrick) {
    double sb = 0.0;
    // bricks blockIdx.x, blockIdx.x + gridDim.x, ... (one each unless there
    // are more than kMaxRedBlocks)
    for (int t = blockIdx.x; t < nbrick; t += gridDim.x) {
        const int i = (t % gx) * blockDim.x + threadIdx.x;
        const int j = ((t / gx) % gy) * blockDim.y + threadIdx.y;
        const int k0 = (t / gx / gy) * kz;
        const int k1 = min(k0 + kz, G.nz);
        if (i >= G.nx || j >= G.ny) continue;
        const size_t plane = (size_t)G.nx * G.ny, col = (size_t)j * G.nx + i;
        const bool side = i == 0 || i == G.nx - 1 || j == 0 || j == G.ny - 1;
        // v = f at (i, j, k); the boundary part is added here
        auto term = [&](int k, double v) -> double {
            const size_t p = (size_t)k * plane + col;
            if (side || k == 0 || k == G.nz - 1) {
                const double be = MODE == COEF_CELL ? eps[p] : 1.0;
                double add = 0.0;
#pragma unroll
                for (int d = 0; d < 6; ++d) {
                    const bool at = d == 0 ? i == 0 : d == 1 ? i == G.nx - 1 : d == 2 ? j == 0
                                  : d == 3 ? j == G.ny - 1 : d == 4 ? k == 0 : k == G.nz - 1;
                    if (at && ((G.bcmask >> d) & 1)) {
                        double bf = be;  // the boundary face's coefficient
                        if constexpr (MODE == COEF_FACE)
                            bf = d == 0 ? face_x(bx, G, i, j, k) : d == 1 ? face_x(bx, G, i + 1, j, k)
                               : d == 2 ? face_y(by, G, i, j, k) : d == 3 ? face_y(by, G, i, j + 1, k)
                               : d == 4 ? face_z(bz, G, i, j, k) : face_z(bz, G, i, j, k + 1);
                        add += 2.0 * bf * G.g[d];
                    }
                }
                v += G.ih2 * add;
            }
            return v * v;
        };
        int k = k0;
        for (; k + 4 <= k1; k += 4) {
            // the four loads are issued before any boundary test needs one
            const double v0 = f[(size_t)k * plane + col], v1 = f[(size_t)(k + 1) * plane + col];
            const double v2 = f[(size_t)(k + 2) * plane + col], v3 = f[(size_t)(k + 3) * plane + col];
            const double t0 = term(k, v0), t1 = term(k + 1, v1), t2 = term(k + 2, v2), t3 = term(k + 3, v3);
            sb += (t0 + t1) + (t2 + t3);
        }
        for (; k < k1; ++k) sb += term(k, f[(size_t)k * plane + col]);
    }
    reduce2_finish<256>(0.0, sb, ws, slot, blockIdx.x);
}
hipError_t norm2_b(hipStream_t s, const Geo &G, const Coef &C, const double *f, const RedWs &ws, int slot) {
    dim3 grid, block;
    int kz;
    brick_shape(G.nx, G.ny, G.nz, kMaxRedBlocks, &grid, &block, &kz);
    const int nbrick = (int)(grid.x * grid.y * grid.z);
    const int nwg = nbrick < kMaxRedBlocks ? nbrick : kMaxRedBlocks;
    const double *eps = (const double *)C.eps, *bx = (const double *)C.bx, *by = (const double *)C.by,
                 *bz = (const double *)C.bz;
    const int gx = (int)grid.x, gy = (int)grid.y;
    switch (C.mode) {
        case COEF_CONST:
            hipLaunchKernelGGL((norm2_b_k<COEF_CONST>), dim3(nwg), block, 0, s, f, eps, bx, by, bz, G, ws, slot, kz,
                               gx, gy, nbrick);
            break;
        case COEF_CELL:
            hipLaunchKernelGGL((norm2_b_k<COEF_CELL>), dim3(nwg), block, 0, s, f, eps, bx, by, bz, G, ws, slot, kz,
                               gx, gy, nbrick);
            break;
        case COEF_FACE:
        case COEF_FACED:
            hipLaunchKernelGGL((norm2_b_k<COEF_FACE>), dim3(nwg), block, 0, s, f, eps, bx, by, bz, G, ws, slot, kz,
                               gx, gy, nbrick);
            break;
        default: return hipErrorInvalidValue;
    }
    if (hipPeekAtLastError() != hipSuccess) return hipGetLastError();
    return reduce2_final(s, ws, slot, slot, nwg, -1, 0.0, nullptr, nullptr);
}
void tile_shape(int t, int *tx, int *ty) {
    static const int TX[kNumTiles + 1] = {0, 64, 128, 64, 32, 32, 16};
    static const int TY[kNumTiles + 1] = {0, 16, 8, 8, 8, 4, 8};
    if (t < 1 || t > kNumTiles) t = 1;
    *tx = TX[t];
    *ty = TY[t];
}

int default_tile(const Geo &G, int st, int mode) {
    (void)st;
    // stored faces keep nine face values per plane in flight: the 64 x 16
    // tile (680 threads, at most 168 registers each) would spill them
    if (!is_face_mode(mode) && G.nx >= 64 && G.ny >= 16 && (long)G.nx * G.ny * G.nz >= (8L << 20))
        return 1;                             // 64 x 16
    if (G.nx >= 64) return 3;                 // 64 x 8
    if (G.nx >= 32) return 4;                 // 32 x 8
    return 6;                                 // 16 x 8
}

int default_zchunk(const Geo &G, int tile, int st, int mode) {
    int tx, ty;
    tile_shape(tile, &tx, &ty);
    const long cols = (long)((G.nx + tx - 1) / tx) * ((G.ny + ty - 1) / ty);
    // about one workgroup per CU (a workgroup holds 5-12 waves) for FP64,
    // two for the FP32/BF16 sweeps, whose smaller register footprint lets
    // two workgroups share a CU and hide each other's per-plane latency
    // (but one where only one fits, which a second round of workgroups would
    // follow: their cell-permittivity sweeps on 64 x 16 tiles, 97-105
    // registers per lane for 11 waves, and their stored-face sweeps on 64 x 8
    // or larger tiles, 153-168 registers for 7 or 11 waves);
    // >= 8 planes per chunk, so the two planes recomputed at each chunk
    // boundary stay a small overhead
    const bool one_per_cu = (mode == COEF_CELL && tx * ty >= 1024) || (is_face_mode(mode) && tx * ty >= 512);
    const long target = (st == ST_F64 || one_per_cu) ? 256 : 512;
    long chunks = (target + cols - 1) / cols;
    long maxchunks = G.nz / 8;
    if (maxchunks < 1) maxchunks = 1;
    if (chunks > maxchunks) chunks = maxchunks;
    if (chunks < 1) chunks = 1;
    return (int)((G.nz + chunks - 1) / chunks);
}

// ------------------------------------------------------------ set-up

__global__ void faces_from_cell_k(const double *__restrict__ eps, double *__restrict__ bx,
                                  double *__restrict__ by, double *__restrict__ bz, Geo G) {
    const int nx = G.nx, ny = G.ny, nz = G.nz;
    const size_t nfx = (size_t)(nx + 1) * ny * nz, nfy = (size_t)nx * (ny + 1) * nz,
                 nfz = (size_t)nx * ny * (nz + 1);
    auto E = [&](int i, int j, int k) { return eps[((size_t)k * ny + j) * nx + i]; };
    auto H = [](double p, double q) { return 2.0 * p * q / (p + q); };
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < nfx + nfy + nfz;
         t += (size_t)gridDim.x * blockDim.x) {
        if (t < nfx) {
            const int i = (int)(t % (nx + 1));
            const size_t r = t / (nx + 1);
            const int j = (int)(r % ny), k = (int)(r / ny);
            bx[t] = i == 0 ? E(0, j, k) : (i == nx ? E(nx - 1, j, k) : H(E(i - 1, j, k), E(i, j, k)));
        } else if (t < nfx + nfy) {
            const size_t u = t - nfx;
            const int i = (int)(u % nx);
            const size_t r = u / nx;
            const int j = (int)(r % (ny + 1)), k = (int)(r / (ny + 1));
            by[u] = j == 0 ? E(i, 0, k) : (j == ny ? E(i, ny - 1, k) : H(E(i, j - 1, k), E(i, j, k)));
        } else {
            const size_t u = t - nfx - nfy;
            const int i = (int)(u % nx);
            const size_t r = u / nx;
            const int j = (int)(r % ny), k = (int)(r / ny);
            bz[u] = k == 0 ? E(i, j, 0) : (k == nz ? E(i, j, nz - 1) : H(E(i, j, k - 1), E(i, j, k)));
        }
    }
}

hipError_t faces_from_cell(hipStream_t s, const Geo &G, const double *eps, double *bx, double *by,
                           double *bz) {
    const size_t n = (size_t)(G.nx + 1) * G.ny * G.nz + (size_t)G.nx * (G.ny + 1) * G.nz +
                     (size_t)G.nx * G.ny * (G.nz + 1);
    size_t g = (n + 255) / 256;
    if (g > 16384) g = 16384;
    hipLaunchKernelGGL(faces_from_cell_k, dim3(g), dim3(256), 0, s, eps, bx, by, bz, G);
    return hipGetLastError();
}

// coarse face = mean of the 4 fine faces it covers
__global__ void coarsen_faces_k(const double *__restrict__ fbx, const double *__restrict__ fby,
                                const double *__restrict__ fbz, Geo Gf, double *__restrict__ cbx,
                                double *__restrict__ cby, double *__restrict__ cbz, Geo Gc) {
    const int nx = Gc.nx, ny = Gc.ny, nz = Gc.nz;
    const int fnx = Gf.nx, fny = Gf.ny;
    const size_t nfx = (size_t)(nx + 1) * ny * nz, nfy = (size_t)nx * (ny + 1) * nz,
                 nfz = (size_t)nx * ny * (nz + 1);
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < nfx + nfy + nfz;
         t += (size_t)gridDim.x * blockDim.x) {
        if (t < nfx) {
            const int i = (int)(t % (nx + 1));
            const size_t r = t / (nx + 1);
            const int j = (int)(r % ny), k = (int)(r / ny);
            double s = 0.0;
            for (int dk = 0; dk < 2; ++dk)
                for (int dj = 0; dj < 2; ++dj)
                    s += fbx[((size_t)(2 * k + dk) * fny + (2 * j + dj)) * (fnx + 1) + 2 * i];
            cbx[t] = 0.25 * s;
        } else if (t < nfx + nfy) {
            const size_t u = t - nfx;
            const int i = (int)(u % nx);
            const size_t r = u / nx;
            const int j = (int)(r % (ny + 1)), k = (int)(r / (ny + 1));
            double s = 0.0;
            for (int dk = 0; dk < 2; ++dk)
                for (int di = 0; di < 2; ++di)
                    s += fby[((size_t)(2 * k + dk) * (fny + 1) + 2 * j) * fnx + (2 * i + di)];
            cby[u] = 0.25 * s;
        } else {
            const size_t u = t - nfx - nfy;
            const int i = (int)(u % nx);
            const size_t r = u / nx;
            const int j = (int)(r % ny), k = (int)(r / ny);
            double s = 0.0;
            for (int dj = 0; dj < 2; ++dj)
                for (int di = 0; di < 2; ++di)
                    s += fbz[((size_t)(2 * k) * fny + (2 * j + dj)) * fnx + (2 * i + di)];
            cbz[u] = 0.25 * s;
        }
    }
}

hipError_t coarsen_faces(hipStream_t s, const Geo &Gf, const double *fbx, const double *fby,
                         const double *fbz, const Geo &Gc, double *cbx, double *cby, double *cbz) {
    const size_t n = (size_t)(Gc.nx + 1) * Gc.ny * Gc.nz + (size_t)Gc.nx * (Gc.ny + 1) * Gc.nz +
                     (size_t)Gc.nx * Gc.ny * (Gc.nz + 1);
    size_t g = (n + 255) / 256;
    if (g > 16384) g = 16384;
    hipLaunchKernelGGL(coarsen_faces_k, dim3(g), dim3(256), 0, s, fbx, fby, fbz, Gf, cbx, cby, cbz,
                       Gc);
    return hipGetLastError();
}

template <class T>
__global__ void convert_k(const double *__restrict__ src, T *__restrict__ dst, size_t n, double factor) {
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (size_t)gridDim.x * blockDim.x)
        dst[t] = Num<T>::cv(typename Num<T>::C(src[t] * factor));
}
template <class T>
__global__ void convert_back_k(const T *__restrict__ src, double *__restrict__ dst, size_t n, double factor) {
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (size_t)gridDim.x * blockDim.x)
        dst[t] = (double)Num<T>::ld(src[t]) * factor;
}
static size_t grid_for(size_t n) {
    size_t g = (n + 255) / 256;
    if (g > 16384) g = 16384;
    if (g < 1) g = 1;
    return g;
}
hipError_t convert(hipStream_t s, const double *src, int st, void *dst, size_t n, double factor) {
    const size_t g = grid_for(n);
    switch (st) {
        case ST_F64:
            hipLaunchKernelGGL(convert_k<double>, dim3(g), dim3(256), 0, s, src, (double *)dst, n, factor);
            break;
        case ST_F32:
            hipLaunchKernelGGL(convert_k<float>, dim3(g), dim3(256), 0, s, src, (float *)dst, n, factor);
            break;
        case ST_BF16:
            hipLaunchKernelGGL(convert_k<bf16>, dim3(g), dim3(256), 0, s, src, (bf16 *)dst, n, factor);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
hipError_t convert_back(hipStream_t s, const void *src, int st, double *dst, size_t n, double factor) {
    const size_t g = grid_for(n);
    switch (st) {
        case ST_F64:
            hipLaunchKernelGGL(convert_back_k<double>, dim3(g), dim3(256), 0, s, (const double *)src, dst, n, factor);
            break;
        case ST_F32:
            hipLaunchKernelGGL(convert_back_k<float>, dim3(g), dim3(256), 0, s, (const float *)src, dst, n, factor);
            break;
        case ST_BF16:
            hipLaunchKernelGGL(convert_back_k<bf16>, dim3(g), dim3(256), 0, s, (const bf16 *)src, dst, n, factor);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
__global__ void scale_f64_k(double *__restrict__ p, size_t n, double factor) {
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (size_t)gridDim.x * blockDim.x)
        p[t] *= factor;
}
hipError_t scale_f64(hipStream_t s, double *p, size_t n, double factor) {
    hipLaunchKernelGGL(scale_f64_k, dim3(grid_for(n)), dim3(256), 0, s, p, n, factor);
    return hipGetLastError();
}
// Largest and smallest entry: per-workgroup partials, then one workgroup.
__global__ __launch_bounds__(256) void minmax_k(const double *__restrict__ x, size_t n, RedWs ws, int slot) {
    __shared__ double sh[2][4];
    double mx = -HUGE_VAL, mn = HUGE_VAL;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (size_t)gridDim.x * blockDim.x) {
        mx = fmax(mx, x[t]);
        mn = fmin(mn, x[t]);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        mx = fmax(mx, __shfl_down(mx, o, 64));
        mn = fmin(mn, __shfl_down(mn, o, 64));
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        sh[0][w] = mx;
        sh[1][w] = mn;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < 4; ++q) {
            mx = fmax(mx, sh[0][q]);
            mn = fmin(mn, sh[1][q]);
        }
        double *part = ws.partials + (size_t)slot * kMaxRedBlocks * 2;
        part[2 * blockIdx.x] = mx;
        part[2 * blockIdx.x + 1] = mn;
    }
}
__global__ __launch_bounds__(64) void minmax_final_k(RedWs ws, int slot, int nb) {
    const double *part = ws.partials + (size_t)slot * kMaxRedBlocks * 2;
    double mx = -HUGE_VAL, mn = HUGE_VAL;
    for (int q = threadIdx.x; q < nb; q += 64) {
        mx = fmax(mx, part[2 * q]);
        mn = fmin(mn, part[2 * q + 1]);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        mx = fmax(mx, __shfl_down(mx, o, 64));
        mn = fmin(mn, __shfl_down(mn, o, 64));
    }
    if (threadIdx.x == 0) {
        ws.result[slot] = mx;
        ws.result[slot + 1] = mn;
    }
}
hipError_t minmax(hipStream_t s, const double *x, size_t n, const RedWs &ws, int slot) {
    size_t g = (n + 255) / 256;
    if (g > (size_t)kMaxRedBlocks) g = kMaxRedBlocks;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(minmax_k, dim3(g), dim3(256), 0, s, x, n, ws, slot);
    if (hipPeekAtLastError() != hipSuccess) return hipGetLastError();
    hipLaunchKernelGGL(minmax_final_k, dim3(1), dim3(64), 0, s, ws, slot, (int)g);
    return hipGetLastError();
}
__global__ __launch_bounds__(256) void count_bad_k(const double *__restrict__ x, size_t n, RedWs ws,
                                                   int slot) {
    double c = 0.0;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (size_t)gridDim.x * blockDim.x) {
        const double v = x[t];
        if (!(v > 0.0 && v <= kMaxCellCoef)) c += 1.0;
    }
    reduce2_finish<256>(c, 0.0, ws, slot, brick_id());
}

hipError_t count_bad(hipStream_t s, const double *x, size_t n, const RedWs &ws, int slot) {
    size_t g = (n + 255) / 256;
    if (g > (size_t)kMaxRedBlocks) g = kMaxRedBlocks;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(count_bad_k, dim3(g), dim3(256), 0, s, x, n, ws, slot);
    if (hipPeekAtLastError() != hipSuccess) return hipGetLastError();
    return reduce2_final(s, ws, slot, -1, (int)g, -1, 0.0, nullptr, nullptr);
}

// Entries outside [lo, hi] (or not finite), counted into ws.result[slot].
__global__ __launch_bounds__(256) void count_outside_k(const double *__restrict__ x, size_t n, double lo,
                                                       double hi, RedWs ws, int slot) {
    double c = 0.0;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
        const double v = x[t];
        if (!(v >= lo && v <= hi)) c += 1.0;
    }
    reduce2_finish<256>(c, 0.0, ws, slot, blockIdx.x);
}

hipError_t count_outside(hipStream_t s, const double *x, size_t n, double lo, double hi, const RedWs &ws,
                         int slot) {
    size_t g = (n + 255) / 256;
    if (g > (size_t)kMaxRedBlocks) g = kMaxRedBlocks;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(count_outside_k, dim3(g), dim3(256), 0, s, x, n, lo, hi, ws, slot);
    if (hipPeekAtLastError() != hipSuccess) return hipGetLastError();
    return reduce2_final(s, ws, slot, -1, (int)g, -1, 0.0, nullptr, nullptr);
}

// Cells whose diagonal a + d + h^-2 (sum of the faces that count) is not
// positive: interior faces, and box faces that are Dirichlet.
__global__ __launch_bounds__(256) void count_singular_k(const double *__restrict__ bx, const double *__restrict__ by,
                                                        const double *__restrict__ bz, const double *__restrict__ d,
                                                        Geo G, RedWs ws, int slot) {
    double c = 0.0;
    const size_t n = (size_t)G.nx * G.ny * G.nz;
    for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(p % G.nx), j = (int)((p / G.nx) % G.ny), k = (int)(p / ((size_t)G.nx * G.ny));
        const bool in[6] = {i > 0, i < G.nx - 1, j > 0, j < G.ny - 1, k > 0, k < G.nz - 1};
        const double f[6] = {face_x(bx, G, i, j, k), face_x(bx, G, i + 1, j, k), face_y(by, G, i, j, k),
                             face_y(by, G, i, j + 1, k), face_z(bz, G, i, j, k), face_z(bz, G, i, j, k + 1)};
        double dg = 0.0;
        for (int q = 0; q < 6; ++q)
            if (in[q] || ((G.bcmask >> q) & 1)) dg += f[q];
        if (!(G.a + d[p] + G.ih2 * dg > 0.0)) c += 1.0;
    }
    reduce2_finish<256>(c, 0.0, ws, slot, blockIdx.x);
}

hipError_t count_singular(hipStream_t s, const Geo &G, const double *bx, const double *by, const double *bz,
                          const double *d, const RedWs &ws, int slot) {
    size_t g = ((size_t)G.nx * G.ny * G.nz + 255) / 256;
    if (g > (size_t)kMaxRedBlocks) g = kMaxRedBlocks;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(count_singular_k, dim3(g), dim3(256), 0, s, bx, by, bz, d, G, ws, slot);
    if (hipPeekAtLastError() != hipSuccess) return hipGetLastError();
    return reduce2_final(s, ws, slot, -1, (int)g, -1, 0.0, nullptr, nullptr);
}

// Coarse cell values: the mean of the 8 children (even fine dimensions).
__global__ void coarsen_cells_k(const double *__restrict__ f, Geo Gf, double *__restrict__ c, Geo Gc) {
    const size_t n = (size_t)Gc.nx * Gc.ny * Gc.nz;
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x) {
        const int I = (int)(q % Gc.nx), J = (int)((q / Gc.nx) % Gc.ny), K = (int)(q / ((size_t)Gc.nx * Gc.ny));
        double s = 0.0;
        for (int o = 0; o < 8; ++o) {
            const size_t p = ((size_t)(2 * K + (o >> 2)) * Gf.ny + (2 * J + ((o >> 1) & 1))) * Gf.nx + 2 * I + (o & 1);
            s += f[p];
        }
        c[q] = 0.125 * s;
    }
}

hipError_t coarsen_cells(hipStream_t s, const Geo &Gf, const double *f, const Geo &Gc, double *c) {
    size_t g = ((size_t)Gc.nx * Gc.ny * Gc.nz + 255) / 256;
    if (g > 16384) g = 16384;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(coarsen_cells_k, dim3(g), dim3(256), 0, s, f, Gf, c, Gc);
    return hipGetLastError();
}

// Zero fill by a kernel (a plain kernel node, safe inside captured graphs).
__global__ void fill_zero_k(uint32_t *__restrict__ p, size_t nwords, uint16_t *tail, int has_tail,
                            const int *__restrict__ done) {
    if (done && *done) return;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < nwords;
         t += (size_t)gridDim.x * blockDim.x)
        p[t] = 0u;
    if (has_tail && blockIdx.x == 0 && threadIdx.x == 0) *tail = 0;
}

hipError_t fill_zero(hipStream_t s, void *p, size_t bytes, const int *done) {
    if (bytes == 0) return hipSuccess;
    const size_t nw = bytes / 4;
    const int has_tail = (bytes % 4) != 0;
    size_t g = (nw + 255) / 256;
    if (g > 16384) g = 16384;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(fill_zero_k, dim3(g), dim3(256), 0, s, (uint32_t *)p, nw,
                       (uint16_t *)((char *)p + nw * 4), has_tail, done);
    return hipGetLastError();
}

__global__ void copy_f64_k(const double *__restrict__ a, double *__restrict__ b, size_t n,
                           const int *__restrict__ done) {
    if (done && *done) return;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (size_t)gridDim.x * blockDim.x)
        b[t] = a[t];
}

hipError_t copy_f64(hipStream_t s, const double *src, double *dst, size_t n, const int *done) {
    size_t g = (n + 255) / 256;
    if (g > 16384) g = 16384;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(copy_f64_k, dim3(g), dim3(256), 0, s, src, dst, n, done);
    return hipGetLastError();
}

// ------------------------------------------------------------ FP64 residual

template <int MODE>
__global__ __launch_bounds__(256) void resid_out_k(const double *__restrict__ u,
                                                   const double *__restrict__ b,
                                                   const double *__restrict__ eps,
                                                   const double *__restrict__ bx,
                                                   const double *__restrict__ by,
                                                   const double *__restrict__ bz, Geo G,
                                                   double *__restrict__ r, const double *__restrict__ dd) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= G.nx || j >= G.ny) return;
    r[((size_t)k * G.ny + j) * G.nx + i] = resid_global<double, MODE>(u, b, eps, bx, by, bz, G, i, j, k, dd);
}

hipError_t resid_out(hipStream_t s, const Geo &G, const Coef &C, const double *u, const double *b,
                     double *r) {
    dim3 grid, block;
    int kz;
    brick_shape(G.nx, G.ny, G.nz, 0, &grid, &block, &kz);
    const double *eps = (const double *)C.eps, *bx = (const double *)C.bx,
                 *by = (const double *)C.by, *bz = (const double *)C.bz;
    switch (C.mode) {
        case COEF_CONST:
            hipLaunchKernelGGL(resid_out_k<COEF_CONST>, grid, block, 0, s, u, b, eps, bx, by, bz, G, r, nullptr);
            break;
        case COEF_CELL:
            hipLaunchKernelGGL(resid_out_k<COEF_CELL>, grid, block, 0, s, u, b, eps, bx, by, bz, G, r, nullptr);
            break;
        case COEF_FACE:
            hipLaunchKernelGGL(resid_out_k<COEF_FACE>, grid, block, 0, s, u, b, eps, bx, by, bz, G, r, nullptr);
            break;
        case COEF_FACED:
            hipLaunchKernelGGL(resid_out_k<COEF_FACED>, grid, block, 0, s, u, b, eps, bx, by, bz, G, r, C.dd);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------ operator apply
// y = alpha x + beta A x, zero boundary values, one thread per cell of a
// brick column (kz planes).
template <int MODE>
__global__ __launch_bounds__(256) void apply_k(const double *__restrict__ x, const double *__restrict__ eps,
                                               const double *__restrict__ bx, const double *__restrict__ by,
                                               const double *__restrict__ bz, Geo G, double alpha, double beta,
                                               double *__restrict__ y, int kz, const double *__restrict__ dd) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k0 = blockIdx.z * kz, k1 = min(k0 + kz, G.nz);
    if (i >= G.nx || j >= G.ny) return;
    const size_t sy = (size_t)G.nx, sz = (size_t)G.nx * G.ny;
    for (int k = k0; k < k1; ++k) {
        const size_t p = (size_t)k * sz + (size_t)j * sy + i;
        auto nb = [&](int d) -> size_t {
            return d == 0 ? p - 1 : d == 1 ? p + 1 : d == 2 ? p - sy : d == 3 ? p + sy : d == 4 ? p - sz : p + sz;
        };
        const double eP = MODE == COEF_CELL ? eps[p] : 1.0;
        double off, dg;
        six_faces<double, MODE>(
            G, i, j, k, eP, [&](int d) { return x[nb(d)]; }, [&](int d) { return eps[nb(d)]; },
            [&](int d) {
                switch (d) {
                    case 0: return face_x(bx, G, i, j, k);
                    case 1: return face_x(bx, G, i + 1, j, k);
                    case 2: return face_y(by, G, i, j, k);
                    case 3: return face_y(by, G, i, j + 1, k);
                    case 4: return face_z(bz, G, i, j, k);
                    default: return face_z(bz, G, i, j, k + 1);
                }
            },
            off, dg);
        const double xP = x[p];
        double ax = G.a * xP + G.ih2 * (dg * xP - off);
        if constexpr (MODE == COEF_FACED) ax += dd[p] * xP;
        y[p] = alpha * xP + beta * ax;
    }
}
// The same for a constant or cell coefficient, marching along z with the
// values of the planes below and above (u, the coefficient and the z face)
// kept in registers: per cell one new u and coefficient load on the axis
// plus the four lateral neighbours, and one new z face.  Every load is
// unconditional (a neighbour outside the box reads the cell itself and is
// masked), so a plane's loads are all in flight together.
template <int MODE>
__global__ __launch_bounds__(256) void apply_z_k(const double *__restrict__ x, const double *__restrict__ eps,
                                                 Geo G, double alpha, double beta, double *__restrict__ y, int kz) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k0 = blockIdx.z * kz, k1 = min(k0 + kz, G.nz);
    if (i >= G.nx || j >= G.ny) return;
    const long sy = G.nx, sz = (long)G.nx * G.ny;
    const bool cell = MODE == COEF_CELL;
    // per-thread neighbour offsets (0 outside the box) and the weights of the
    // lateral boundary faces (2 on a Dirichlet face, else 0)
    const bool in[4] = {i > 0, i < G.nx - 1, j > 0, j < G.ny - 1};
    const long off4[4] = {in[0] ? -1 : 0, in[1] ? 1 : 0, in[2] ? -sy : 0, in[3] ? sy : 0};
    double bw = 0.0;
#pragma unroll
    for (int d = 0; d < 4; ++d)
        if (!in[d] && ((G.bcmask >> d) & 1)) bw += 2.0;
    const double bz0 = ((G.bcmask >> 4) & 1) ? 2.0 : 0.0, bz1 = ((G.bcmask >> 5) & 1) ? 2.0 : 0.0;
    long p = (long)k0 * sz + (long)j * sy + i;
    double xc = x[p], ec = cell ? eps[p] : 1.0;
    double xm = 0.0, fm = bz0 * ec;  // the face below: a Dirichlet domain face or none
    if (k0 > 0) {
        xm = x[p - sz];
        fm = cell ? harm_face(ec, eps[p - sz]) : 1.0;
    }
    for (int k = k0; k < k1; ++k, p += sz) {
        const bool up = k < G.nz - 1;
        const long pu = up ? p + sz : p;
        double xn[4], en[4];
#pragma unroll
        for (int d = 0; d < 4; ++d) xn[d] = x[p + off4[d]];
        const double xp_raw = x[pu];
        const double ep_raw = cell ? eps[pu] : 1.0;
        if (cell) {
#pragma unroll
            for (int d = 0; d < 4; ++d) en[d] = eps[p + off4[d]];
        }
        const double xp = up ? xp_raw : 0.0;
        const double fp = up ? (cell ? harm_face(ec, ep_raw) : 1.0) : bz1 * ec;
        double off = fm * xm + fp * xp, dg = fm + fp + bw * ec;
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const double f = in[d] ? (cell ? harm_face(ec, en[d]) : 1.0) : 0.0;
            off += f * xn[d];
            dg += f;
        }
        const double ax = G.a * xc + G.ih2 * (dg * xc - off);
        y[p] = alpha * xc + beta * ax;
        xm = xc;
        xc = xp;
        fm = fp;
        ec = up ? ep_raw : ec;
    }
}

hipError_t apply_op(hipStream_t s, const Geo &G0, const Coef &C, double alpha, double beta, const double *x,
                    double *y) {
    Geo G = G0;
    for (int d = 0; d < 6; ++d) G.g[d] = 0.0;
    dim3 grid, block;
    int kz;
    brick_shape(G.nx, G.ny, G.nz, 4096, &grid, &block, &kz);
    const double *eps = (const double *)C.eps, *bx = (const double *)C.bx, *by = (const double *)C.by,
                 *bz = (const double *)C.bz;
    switch (C.mode) {
        case COEF_CONST:
            hipLaunchKernelGGL(apply_z_k<COEF_CONST>, grid, block, 0, s, x, eps, G, alpha, beta, y, kz);
            break;
        case COEF_CELL:
            hipLaunchKernelGGL(apply_z_k<COEF_CELL>, grid, block, 0, s, x, eps, G, alpha, beta, y, kz);
            break;
        case COEF_FACE:
            hipLaunchKernelGGL(apply_k<COEF_FACE>, grid, block, 0, s, x, eps, bx, by, bz, G, alpha, beta, y, kz,
                               nullptr);
            break;
        case COEF_FACED:
            hipLaunchKernelGGL(apply_k<COEF_FACED>, grid, block, 0, s, x, eps, bx, by, bz, G, alpha, beta, y, kz,
                               C.dd);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------ field
// E = -grad(phi) by central differences, |E| and sigma |E| maximised per
// workgroup (partials of ws slot `slot`, then field_final_k).  Bricks as
// norm2_b_k.
__global__ __launch_bounds__(256) void field_k(const double *__restrict__ phi, const double *__restrict__ sigma,
                                               Geo G, double inv2h, double *__restrict__ ex,
                                               double *__restrict__ ey, double *__restrict__ ez, RedWs ws,
                                               int slot, int kz, int gx, int gy, int nbrick) {
    double me = 0.0, mj = 0.0;
    const size_t sy = (size_t)G.nx, sz = (size_t)G.nx * G.ny;
    for (int t = blockIdx.x; t < nbrick; t += gridDim.x) {
        const int i = (t % gx) * blockDim.x + threadIdx.x;
        const int j = ((t / gx) % gy) * blockDim.y + threadIdx.y;
        const int k0 = (t / gx / gy) * kz, k1 = min(k0 + kz, G.nz);
        if (i >= G.nx || j >= G.ny) continue;
        for (int k = k0; k < k1; ++k) {
            const size_t p = (size_t)k * sz + (size_t)j * sy + i;
            const double u = phi[p];
            // neighbour or ghost value in direction d
            auto nb = [&](int d, bool in, size_t q) -> double {
                if (in) return phi[q];
                return ((G.bcmask >> d) & 1) ? 2.0 * G.g[d] - u : u;
            };
            const double xm = nb(0, i > 0, p - 1), xp = nb(1, i < G.nx - 1, p + 1);
            const double ym = nb(2, j > 0, p - sy), yp = nb(3, j < G.ny - 1, p + sy);
            const double zm = nb(4, k > 0, p - sz), zp = nb(5, k < G.nz - 1, p + sz);
            const double fx = (xm - xp) * inv2h, fy = (ym - yp) * inv2h, fz = (zm - zp) * inv2h;
            if (ex) ex[p] = fx;
            if (ey) ey[p] = fy;
            if (ez) ez[p] = fz;
            const double e = sqrt(fx * fx + fy * fy + fz * fz);
            me = fmax(me, e);
            if (sigma) mj = fmax(mj, sigma[p] * e);
        }
    }
    __shared__ double sh[2][4];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        me = fmax(me, __shfl_down(me, o, 64));
        mj = fmax(mj, __shfl_down(mj, o, 64));
    }
    const int tid = threadIdx.x + blockDim.x * threadIdx.y, lane = tid & 63, w = tid >> 6;
    if (lane == 0) {
        sh[0][w] = me;
        sh[1][w] = mj;
    }
    __syncthreads();
    if (tid == 0) {
        for (int q = 1; q < 4; ++q) {
            me = fmax(me, sh[0][q]);
            mj = fmax(mj, sh[1][q]);
        }
        double *part = ws.partials + (size_t)slot * kMaxRedBlocks * 2;
        part[2 * blockIdx.x] = me;
        part[2 * blockIdx.x + 1] = mj;
    }
}
__global__ __launch_bounds__(64) void field_final_k(RedWs ws, int slot, int nb) {
    const double *part = ws.partials + (size_t)slot * kMaxRedBlocks * 2;
    double me = 0.0, mj = 0.0;
    for (int q = threadIdx.x; q < nb; q += 64) {
        me = fmax(me, part[2 * q]);
        mj = fmax(mj, part[2 * q + 1]);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        me = fmax(me, __shfl_down(me, o, 64));
        mj = fmax(mj, __shfl_down(mj, o, 64));
    }
    if (threadIdx.x == 0) {
        ws.result[slot] = me;
        ws.result[slot + 1] = mj;
    }
}
hipError_t field(hipStream_t s, const Geo &G, double h, const double *phi, const double *sigma, double *ex,
                 double *ey, double *ez, const RedWs &ws, int slot) {
    dim3 grid, block;
    int kz;
    brick_shape(G.nx, G.ny, G.nz, kMaxRedBlocks, &grid, &block, &kz);
    const int nbrick = (int)(grid.x * grid.y * grid.z);
    const int nwg = nbrick < kMaxRedBlocks ? nbrick : kMaxRedBlocks;
    hipLaunchKernelGGL(field_k, dim3(nwg), block, 0, s, phi, sigma, G, 0.5 / h, ex, ey, ez, ws, slot, kz,
                       (int)grid.x, (int)grid.y, nbrick);
    if (hipPeekAtLastError() != hipSuccess) return hipGetLastError();
    hipLaunchKernelGGL(field_final_k, dim3(1), dim3(64), 0, s, ws, slot, nwg);
    return hipGetLastError();
}

// ------------------------------------------------------------ refinement
template <class TL, int MODE, bool HAS_E, int TX, int TY>
__global__ __launch_bounds__(TX *TY) void ir_col_k(const double *__restrict__ x, const TL *__restrict__ e,
                                                   double *__restrict__ xout, const double *__restrict__ b,
                                                   const double *__restrict__ eps, Geo G, TL *__restrict__ rl,
                                                   RedWs ws, int slot, int cz, int tiles_x, int tiles_y,
                                                   int nblk, double sc0, double cs,
                                                   const int *__restrict__ done_in) {
    if (done_in && *done_in) return;
    ir_tiles<TL, MODE, HAS_E, TX, TY, true>(x, e, xout, b, eps, G, rl, ws, slot, -1, cz, tiles_x, tiles_y,
                                            blockIdx.x, nblk, gridDim.x, xcd_remap(blockIdx.x, gridDim.x), false,
                                            ws.result + kSlotScale, sc0, cs);
}
__global__ __launch_bounds__(kFinalThreads) void ir_final_k(RedWs ws, int slot, int nb, int ref_slot, double rtol2,
                                                            int *done, const int *done_in, double sc0, double n) {
    if (done_in && *done_in) return;
    ir_final_body(ws, slot, -1, nb, ref_slot, rtol2, done, ws.result + kSlotScale, sc0, n);
}
template <class TL>
static hipError_t ir_update_resid_T(hipStream_t s, const Geo &G, const Coef &C, const double *x,
                                    const void *e, double *xout, const double *b, void *r_lp,
                                    const RrCheck &k, double sc0, double cs) {
    constexpr int TX = 64, TY = 4;
    const int tiles_x = (G.nx + TX - 1) / TX, tiles_y = (G.ny + TY - 1) / TY;
    // about kMaxRedBlocks tiles (z chunks of the column tiles); planes wider
    // than that many column tiles make each workgroup cover several tiles
    int chunks = kMaxRedBlocks / (tiles_x * tiles_y);
    if (chunks < 1) chunks = 1;
    if (chunks > G.nz) chunks = G.nz;
    const int cz = (G.nz + chunks - 1) / chunks;
    chunks = (G.nz + cz - 1) / cz;
    const int nblk = tiles_x * tiles_y * chunks;
    const int nwg = nblk < kMaxRedBlocks ? nblk : kMaxRedBlocks;
    const double *eps = (const double *)C.eps;
    const TL *el = (const TL *)e;
    TL *rl = (TL *)r_lp;
#define MG_IR_LAUNCH(MODE, HE)                                                                                   \
    hipLaunchKernelGGL((ir_col_k<TL, MODE, HE, TX, TY>), dim3(nwg), dim3(TX * TY), 0, s, x, el, xout, b, eps, G,  \
                       rl, k.ws, k.slot, cz, tiles_x, tiles_y, nblk, sc0, cs, k.done_in)
    if (C.mode == COEF_CELL) {
        if (e) MG_IR_LAUNCH(COEF_CELL, true);
        else MG_IR_LAUNCH(COEF_CELL, false);
    } else if (C.mode == COEF_CONST) {
        if (e) MG_IR_LAUNCH(COEF_CONST, true);
        else MG_IR_LAUNCH(COEF_CONST, false);
    } else {
        return hipErrorInvalidValue;
    }
#undef MG_IR_LAUNCH
    if (hipPeekAtLastError() != hipSuccess) return hipGetLastError();
    hipLaunchKernelGGL(ir_final_k, dim3(1), dim3(kFinalThreads), 0, s, k.ws, k.slot, nwg, k.ref_slot, k.rtol2,
                       k.done_out, k.done_in, sc0, (double)G.nx * G.ny * G.nz);
    return hipGetLastError();
}
hipError_t ir_update_resid(hipStream_t s, const Geo &G, const Coef &C, const double *x,
                           const void *e, double *xout, const double *b, int stl, void *r_lp,
                           const RrCheck &chk, double sc0, double cs) {
    switch (stl) {
        case ST_F32: return ir_update_resid_T<float>(s, G, C, x, e, xout, b, r_lp, chk, sc0, cs);
        case ST_BF16: return ir_update_resid_T<bf16>(s, G, C, x, e, xout, b, r_lp, chk, sc0, cs);
    }
    return hipErrorInvalidValue;
}

}  // namespace mg
