// Embedded-boundary (cut-cell) solves: the C ABI of mge.h.
//
// The cut-cell operator is applied by one z-marching kernel over every cell
// (aperture-weighted faces, covered cells as identity rows) plus a kernel
// over the boundary cells that adds the embedded face's flux through a
// precomputed 16-point stencil (two trilinear interpolations along the
// normal ray).  The stencils are built on the device at set-up from the
// apertures and the surface points.  BiCGStab (mg_krylov) solves the
// non-symmetric system with one engine V-cycle per preconditioner call on
// the symmetric part of the cut-cell operator: the aperture-weighted faces,
// the diagonal of the embedded face's stencil (its 1.5 beta A / h^2 at the
// surface) and identity rows for covered cells, set up through
// mg_set_face_coeffs_diag.  Covered cells are fixed at the electrode
// potential from the start and the preconditioner's output is zero there,
// so their rows stay satisfied.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "mg_engine.h"
#include "mg_krylov.h"
#include "mg_stencil.cuh"
#include "mge.h"

namespace mg {

struct EbGeo {
    int nx, ny, nz;
    double h, ih2, a;
    int bcmask;
    double g[6];  // box-face values (0 in the operator apply)
};

constexpr int kEbStencil = 16;             // two trilinear interpolations

namespace {

// One cell's row of the regular part.  Neighbour offsets are 0 across the
// box faces (the loads then read the cell itself and are masked).
template <bool RHS>
__global__ __launch_bounds__(256) void eb_apply_k(const double *__restrict__ x, const double *__restrict__ f,
                                                  const double *__restrict__ eps, const double *__restrict__ kappa,
                                                  const double *__restrict__ ax, const double *__restrict__ ay,
                                                  const double *__restrict__ az, const double *__restrict__ gc,
                                                  double g_eb, EbGeo G, double *__restrict__ y, int kz) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k0 = blockIdx.z * kz, k1 = min(k0 + kz, G.nz);
    if (i >= G.nx || j >= G.ny) return;
    const long sy = G.nx, sz = (long)G.nx * G.ny;
    const long sxf = G.nx + 1;  // row length of ax
    const bool in[4] = {i > 0, i < G.nx - 1, j > 0, j < G.ny - 1};
    const long off4[4] = {in[0] ? -1 : 0, in[1] ? 1 : 0, in[2] ? -sy : 0, in[3] ? sy : 0};
    const bool dir[6] = {((G.bcmask >> 0) & 1) != 0, ((G.bcmask >> 1) & 1) != 0, ((G.bcmask >> 2) & 1) != 0,
                         ((G.bcmask >> 3) & 1) != 0, ((G.bcmask >> 4) & 1) != 0, ((G.bcmask >> 5) & 1) != 0};
    for (int k = k0; k < k1; ++k) {
        const long p = (long)k * sz + (long)j * sy + i;
        const bool dn = k > 0, up = k < G.nz - 1;
        const double kp = kappa[p];
        const double eP = eps ? eps[p] : 1.0;
        // apertures of the six faces
        const long fxp = ((long)k * G.ny + j) * sxf + i;
        const long fyp = ((long)k * (G.ny + 1) + j) * G.nx + i;
        const double al[6] = {ax[fxp], ax[fxp + 1], ay[fyp], ay[fyp + G.nx], az[p], az[p + sz]};
        const long offs[6] = {off4[0], off4[1], off4[2], off4[3], dn ? -sz : 0, up ? sz : 0};
        const bool inb[6] = {in[0], in[1], in[2], in[3], dn, up};
        double off = 0.0, dg = 0.0, bnd = 0.0;
#pragma unroll
        for (int d = 0; d < 6; ++d) {
            const double xn = RHS ? 0.0 : x[p + offs[d]];
            const double en = eps ? eps[p + offs[d]] : 1.0;
            if (inb[d]) {
                const double c = harm_face(eP, en) * al[d];
                off += c * xn;
                dg += c;
            } else if (dir[d]) {
                const double c = 2.0 * eP * al[d];
                dg += c;
                bnd += c * G.g[d];
            }
        }
        double out;
        if (kp <= 0.0) {
            out = RHS ? G.ih2 * (gc ? gc[p] : g_eb) : G.ih2 * x[p];
        } else if (RHS) {
            out = kp * f[p] + G.ih2 * bnd;
        } else {
            const double xP = x[p];
            out = kp * G.a * xP + G.ih2 * (dg * xP - off);
        }
        y[p] = out;
    }
}

// Boundary cells: y_P += sum of the embedded-face stencil times x.
__global__ __launch_bounds__(256) void eb_fix_k(const double *__restrict__ x, double *__restrict__ y,
                                                const long *__restrict__ bidx, const long *__restrict__ sidx,
                                                const double *__restrict__ sw, long nb) {
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < nb; q += (long)gridDim.x * blockDim.x) {
        double acc = 0.0;
#pragma unroll
        for (int m = 0; m < kEbStencil; ++m) acc += sw[q * kEbStencil + m] * x[sidx[q * kEbStencil + m]];
        y[bidx[q]] += acc;
    }
}

// Boundary cells of the right-hand side: + 1.5 coef g_P.
__global__ void eb_rhs_fix_k(double *__restrict__ b, const long *__restrict__ bidx, const double *__restrict__ c15,
                             const double *__restrict__ gc, double g_eb, long nb) {
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < nb; q += (long)gridDim.x * blockDim.x) {
        const long p = bidx[q];
        b[p] += c15[q] * (gc ? gc[p] : g_eb);
    }
}

// The embedded face of each boundary cell: area vector from the apertures
// (A n = -sum alpha_f n_f), inward normal nu = -n, and the stencil of
// beta A / h^2 (2 u(x_b + h nu) - u(x_b + 2 h nu) / 2), each point valued
// by trilinear interpolation of the 8 surrounding cell centres (the block
// shifted inside the box where needed).
__global__ void eb_setup_k(const long *__restrict__ bidx, const double *__restrict__ boff,
                           const double *__restrict__ eps, const double *__restrict__ ax,
                           const double *__restrict__ ay, const double *__restrict__ az, EbGeo G, long nb,
                           long *__restrict__ sidx, double *__restrict__ sw, double *__restrict__ c15,
                           double *__restrict__ pc_diag) {
    const long sz = (long)G.nx * G.ny;
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < nb; q += (long)gridDim.x * blockDim.x) {
        const long p = bidx[q];
        const int i = (int)(p % G.nx), j = (int)((p / G.nx) % G.ny), k = (int)(p / sz);
        const long fxp = ((long)k * G.ny + j) * (G.nx + 1) + i;
        const long fyp = ((long)k * (G.ny + 1) + j) * G.nx + i;
        const double an[3] = {-(ax[fxp + 1] - ax[fxp]), -(ay[fyp + G.nx] - ay[fyp]), -(az[p + sz] - az[p])};
        const double A = sqrt(an[0] * an[0] + an[1] * an[1] + an[2] * an[2]);
        double nu[3] = {0.0, 0.0, 0.0};
        if (A > 1e-12)
            for (int d = 0; d < 3; ++d) nu[d] = -an[d] / A;
        const double eP = eps ? eps[p] : 1.0;
        const double coef = eP * A * G.ih2;
        const double del[3] = {boff[3 * q], boff[3 * q + 1], boff[3 * q + 2]};
        const double xb[3] = {i + 0.5 + del[0], j + 0.5 + del[1], k + 0.5 + del[2]};
        const int dims[3] = {G.nx, G.ny, G.nz};
        for (int m = 0; m < 2; ++m) {
            const double dist = m + 1.0, scale = m == 0 ? 2.0 * coef : -0.5 * coef;
            int lo[3];
            double t[3];
            for (int d = 0; d < 3; ++d) {
                // (clamped before the conversion: the block is shifted inside the box anyway)
                const double c = fmin(fmax(xb[d] + dist * nu[d] - 0.5, -1.0), (double)dims[d]);
                int l = (int)floor(c);
                l = l < 0 ? 0 : (l > dims[d] - 2 ? dims[d] - 2 : l);
                lo[d] = l;
                t[d] = c - l;
            }
            for (int o = 0; o < 8; ++o) {
                const int ox = o & 1, oy = (o >> 1) & 1, oz = o >> 2;
                const double wx = ox ? t[0] : 1.0 - t[0];
                const double wy = oy ? t[1] : 1.0 - t[1];
                const double wz = oz ? t[2] : 1.0 - t[2];
                const long e = q * kEbStencil + m * 8 + o;
                sidx[e] = ((long)(lo[2] + oz) * G.ny + (lo[1] + oy)) * G.nx + (lo[0] + ox);
                sw[e] = scale * (wx * wy * wz);
            }
        }
        c15[q] = 1.5 * coef;
        pc_diag[p] += 1.5 * coef;  // the stencil's weight at the surface point
    }
}

// The preconditioner's face coefficients: aperture times the harmonic
// beta inside, aperture times the cell's beta on the box faces.
__global__ void eb_pc_faces_k(const double *__restrict__ ax, const double *__restrict__ ay,
                              const double *__restrict__ az, const double *__restrict__ eps, EbGeo G,
                              double *__restrict__ bx, double *__restrict__ by, double *__restrict__ bz) {
    const long nfx = (long)(G.nx + 1) * G.ny * G.nz, nfy = (long)G.nx * (G.ny + 1) * G.nz;
    const long nfz = (long)G.nx * G.ny * (G.nz + 1), sz = (long)G.nx * G.ny;
    auto beta = [&](long p) { return eps ? eps[p] : 1.0; };
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < nfx + nfy + nfz;
         q += (long)gridDim.x * blockDim.x) {
        if (q < nfx) {
            const int i = (int)(q % (G.nx + 1));
            const long row = q / (G.nx + 1);  // k * ny + j
            const long p = row * G.nx + i;    // the cell above the face (i), if any
            const double b = i == 0 ? beta(p) : i == G.nx ? beta(p - 1) : harm_face(beta(p - 1), beta(p));
            bx[q] = ax[q] * b;
        } else if (q < nfx + nfy) {
            const long t = q - nfx;
            const int i = (int)(t % G.nx), j = (int)((t / G.nx) % (G.ny + 1));
            const long k = t / ((long)G.nx * (G.ny + 1));
            const long p = (k * G.ny + j) * G.nx + i;
            const double b = j == 0 ? beta(p) : j == G.ny ? beta(p - G.nx) : harm_face(beta(p - G.nx), beta(p));
            by[t] = ay[t] * b;
        } else {
            const long t = q - nfx - nfy;
            const long k = t / sz;
            const double b = k == 0 ? beta(t) : k == G.nz ? beta(t - sz) : harm_face(beta(t - sz), beta(t));
            bz[t] = az[t] * b;
        }
    }
}

// The preconditioner's diagonal: kappa a, or 1 / h^2 on covered cells; the
// embedded faces add theirs in eb_setup_k.
__global__ void eb_pc_diag_k(const double *__restrict__ kappa, EbGeo G, double *__restrict__ d, long n) {
    for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (long)gridDim.x * blockDim.x)
        d[p] = kappa[p] <= 0.0 ? G.ih2 : kappa[p] * G.a;
}

__global__ void eb_set_list_k(double *__restrict__ v, const long *__restrict__ list, long m,
                              const double *__restrict__ gc, double val) {
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < m; q += (long)gridDim.x * blockDim.x) {
        const long p = list[q];
        v[p] = gc ? gc[p] : val;
    }
}

// partial count of entries outside [lo, hi] (or not finite)
__global__ __launch_bounds__(256) void eb_range_k(const double *__restrict__ x, long n, double lo, double hi,
                                                  RedWs ws, int slot) {
    double c = 0.0;
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
        const double v = x[t];
        if (!(v >= lo && v <= hi)) c += 1.0;
    }
    reduce2_finish<256>(c, 0.0, ws, slot, blockIdx.x);
}

unsigned grid1(long n) { return (unsigned)std::min<long>(std::max<long>((n + 255) / 256, 1), 16384); }

}  // namespace
}  // namespace mg

struct mge_ctx {
    mg_desc d{};
    hipStream_t stream = nullptr;
    mg::EbGeo G{};
    long n = 0, nb = 0, ncov = 0;
    double *kappa = nullptr, *ax = nullptr, *ay = nullptr, *az = nullptr, *eps = nullptr, *gc = nullptr;
    double g_eb = 0.0;
    long *bidx = nullptr, *cov = nullptr, *sidx = nullptr;
    double *sw = nullptr, *c15 = nullptr;
    double *b = nullptr;  // right-hand side
    mg::KrylovSpace K;
    mg_ctx *pc = nullptr;  // the preconditioner's regular-grid operator
    bool ready = false;
};

using namespace mg;

namespace {

#define ECK(expr)                                                                                  \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return set_err(MG_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),       \
                           __FILE__, __LINE__);                                                    \
    } while (0)

void free_geometry(mge_ctx *e) {
    for (double **p : {&e->kappa, &e->ax, &e->ay, &e->az, &e->eps, &e->gc, &e->sw, &e->c15})
        if (*p) {
            (void)hipFree(*p);
            *p = nullptr;
        }
    for (long **p : {&e->bidx, &e->cov, &e->sidx})
        if (*p) {
            (void)hipFree(*p);
            *p = nullptr;
        }
    e->nb = e->ncov = 0;
    e->ready = false;
}

int apply(mge_ctx *e, const double *x, double *y) {
    dim3 grid, block;
    int kz;
    brick_shape(e->G.nx, e->G.ny, e->G.nz, 4096, &grid, &block, &kz);
    EbGeo G = e->G;
    for (int f = 0; f < 6; ++f) G.g[f] = 0.0;
    hipLaunchKernelGGL(eb_apply_k<false>, grid, block, 0, e->stream, x, nullptr, e->eps, e->kappa, e->ax, e->ay,
                       e->az, nullptr, 0.0, G, y, kz);
    ECK(hipGetLastError());
    if (e->nb > 0) {
        hipLaunchKernelGGL(eb_fix_k, dim3(grid1(e->nb)), dim3(256), 0, e->stream, x, y, e->bidx, e->sidx, e->sw,
                           e->nb);
        ECK(hipGetLastError());
    }
    return MG_OK;
}

int rhs(mge_ctx *e, const double *f, double *b) {
    dim3 grid, block;
    int kz;
    brick_shape(e->G.nx, e->G.ny, e->G.nz, 4096, &grid, &block, &kz);
    hipLaunchKernelGGL(eb_apply_k<true>, grid, block, 0, e->stream, nullptr, f, e->eps, e->kappa, e->ax, e->ay,
                       e->az, e->gc, e->g_eb, e->G, b, kz);
    ECK(hipGetLastError());
    if (e->nb > 0) {
        hipLaunchKernelGGL(eb_rhs_fix_k, dim3(grid1(e->nb)), dim3(256), 0, e->stream, b, e->bidx, e->c15, e->gc,
                           e->g_eb, e->nb);
        ECK(hipGetLastError());
    }
    return MG_OK;
}

// z = M^-1 v: one V-cycle of the regular-grid operator, zero on covered cells
int precond(mge_ctx *e, const double *v, double *z) {
    std::vector<LvView> V;
    fp64_view(e->pc, V, v, z);
    if (int rc = vcycle(e->pc, V, 0, true)) return rc;
    if (V[0].u != z) ECK(hipMemcpyAsync(z, V[0].u, e->n * 8, hipMemcpyDeviceToDevice, e->stream));
    if (e->ncov > 0) {
        hipLaunchKernelGGL(eb_set_list_k, dim3(grid1(e->ncov)), dim3(256), 0, e->stream, z, e->cov, e->ncov,
                           nullptr, 0.0);
        ECK(hipGetLastError());
    }
    return MG_OK;
}

// number of entries of x outside [lo, hi] (device array)
int count_outside(mge_ctx *e, const double *x, long n, double lo, double hi, double *out) {
    const unsigned nb = std::min<unsigned>(grid1(n), kMaxRedBlocks);
    hipLaunchKernelGGL(eb_range_k, dim3(nb), dim3(256), 0, e->stream, x, n, lo, hi, e->K.ws, 0);
    ECK(hipGetLastError());
    ECK(reduce2_final(e->stream, e->K.ws, 0, -1, (int)nb, -1, 0.0, nullptr, nullptr));
    ECK(hipMemcpyAsync(e->K.h_pin, e->K.ws.result, sizeof(double), hipMemcpyDeviceToHost, e->stream));
    ECK(hipStreamSynchronize(e->stream));
    *out = e->K.h_pin[0];
    return MG_OK;
}

}  // namespace

extern "C" {

int mge_destroy(mge_ctx *e) {
    if (!e) return MG_OK;
    (void)hipStreamSynchronize(e->stream);
    free_geometry(e);
    if (e->b) (void)hipFree(e->b);
    if (e->pc) mg_destroy(e->pc);
    krylov_free(e->K);
    delete e;
    return MG_OK;
}

int mge_create(const mg_desc *d, void *hip_stream, mge_ctx **out) {
    if (out) *out = nullptr;
    if (!d || !out) return set_err(MG_EINVAL, "mge_create: null argument");
    if (d->precision != MG_FP64) return set_err(MG_EINVAL, "mge_create: cut-cell solves run in MG_FP64");
    if (int rc = check_grid("mge_create", d)) return rc;
    if (d->nx < 2 || d->ny < 2 || d->nz < 2) return set_err(MG_EINVAL, "mge_create: every axis needs >= 2 cells");
    mge_ctx *e = new mge_ctx();
    e->d = *d;
    e->stream = (hipStream_t)hip_stream;
    e->n = (long)d->nx * d->ny * d->nz;
    e->G.nx = d->nx;
    e->G.ny = d->ny;
    e->G.nz = d->nz;
    e->G.h = d->h;
    e->G.ih2 = 1.0 / (d->h * d->h);
    int rc = mg_create(d, hip_stream, &e->pc);
    if (rc == MG_OK) rc = krylov_alloc(e->K, e->stream, e->n, e->n, 1.0);
    if (rc == MG_OK && hipMalloc(&e->b, sizeof(double) * e->n) != hipSuccess)
        rc = set_err(MG_ENOMEM, "mge_create: device allocation failed");
    if (rc != MG_OK) {
        mge_destroy(e);
        return rc;
    }
    *out = e;
    return MG_OK;
}

int mge_set_geometry(mge_ctx *e, const double *kappa, const double *ax, const double *ay, const double *az,
                     long nb, const long *bidx, const double *boff, const double *eps, double a, const mg_bcs *bc,
                     const double *g, double g_eb) {
    if (!e || !kappa || !ax || !ay || !az || !bc || nb < 0 || (nb > 0 && (!bidx || !boff)))
        return set_err(MG_EINVAL, "mge_set_geometry: null argument");
    int mask = 0;
    if (int rc = parse_operator("mge_set_geometry", a, bc, &mask)) return rc;
    if (!std::isfinite(g_eb)) return set_err(MG_EINVAL, "mge_set_geometry: g_eb is not finite");
    free_geometry(e);
    const long n = e->n, nx = e->G.nx, ny = e->G.ny, nz = e->G.nz;
    const long nfx = (nx + 1) * ny * nz, nfy = nx * (ny + 1) * nz, nfz = nx * ny * (nz + 1);
    hipStream_t s = e->stream;
    bool ok = hipMalloc(&e->kappa, 8 * n) == hipSuccess && hipMalloc(&e->ax, 8 * nfx) == hipSuccess &&
              hipMalloc(&e->ay, 8 * nfy) == hipSuccess && hipMalloc(&e->az, 8 * nfz) == hipSuccess &&
              (!eps || hipMalloc(&e->eps, 8 * n) == hipSuccess) &&
              (!g || hipMalloc(&e->gc, 8 * n) == hipSuccess) &&
              hipMalloc(&e->bidx, 8 * std::max<long>(nb, 1)) == hipSuccess &&
              hipMalloc(&e->sidx, 8 * kEbStencil * std::max<long>(nb, 1)) == hipSuccess &&
              hipMalloc(&e->sw, 8 * kEbStencil * std::max<long>(nb, 1)) == hipSuccess &&
              hipMalloc(&e->c15, 8 * std::max<long>(nb, 1)) == hipSuccess;
    if (!ok) {
        free_geometry(e);
        return set_err(MG_ENOMEM, "mge_set_geometry: device allocation failed");
    }
    ECK(hipMemcpyAsync(e->kappa, kappa, 8 * n, hipMemcpyDeviceToDevice, s));
    ECK(hipMemcpyAsync(e->ax, ax, 8 * nfx, hipMemcpyDeviceToDevice, s));
    ECK(hipMemcpyAsync(e->ay, ay, 8 * nfy, hipMemcpyDeviceToDevice, s));
    ECK(hipMemcpyAsync(e->az, az, 8 * nfz, hipMemcpyDeviceToDevice, s));
    if (eps) ECK(hipMemcpyAsync(e->eps, eps, 8 * n, hipMemcpyDeviceToDevice, s));
    if (g) ECK(hipMemcpyAsync(e->gc, g, 8 * n, hipMemcpyDeviceToDevice, s));
    // value ranges, checked on the device
    struct Chk { const double *p; long n; double lo, hi; const char *name; };
    const Chk chks[] = {{e->kappa, n, 0.0, 1.0, "kappa"}, {e->ax, nfx, 0.0, 1.0, "ax"}, {e->ay, nfy, 0.0, 1.0, "ay"},
                        {e->az, nfz, 0.0, 1.0, "az"}, {e->eps, n, 1e-300, 1e96, "eps"},
                        {e->gc, n, -1e300, 1e300, "g"}};
    for (const Chk &c : chks) {
        if (!c.p) continue;
        double bad = 0.0;
        if (int rc = count_outside(e, c.p, c.n, c.lo, c.hi, &bad)) return rc;
        if (bad != 0.0) {
            free_geometry(e);
            return set_err(MG_EINVAL, "mge_set_geometry: %.0f entries of %s out of range", bad, c.name);
        }
    }
    // host checks of the boundary list; the covered list from kappa
    std::vector<double> hk(n);
    ECK(hipMemcpy(hk.data(), e->kappa, 8 * n, hipMemcpyDeviceToHost));
    for (long q = 0; q < nb; ++q) {
        const long p = bidx[q];
        const bool bad = p < 0 || p >= n || (q > 0 && p <= bidx[q - 1]) || !(hk[p] > 0.0) ||
                         !std::isfinite(boff[3 * q]) || !std::isfinite(boff[3 * q + 1]) ||
                         !std::isfinite(boff[3 * q + 2]);
        if (bad) {
            free_geometry(e);
            return set_err(MG_EINVAL,
                           "mge_set_geometry: boundary cell %ld (index %ld) is out of order, outside the grid, "
                           "covered, or has a non-finite surface point",
                           q, p);
        }
    }
    std::vector<long> cov;
    for (long p = 0; p < n; ++p)
        if (hk[p] <= 0.0) cov.push_back(p);
    e->ncov = (long)cov.size();
    if (e->ncov > 0) {
        if (hipMalloc(&e->cov, 8 * e->ncov) != hipSuccess) {
            free_geometry(e);
            return set_err(MG_ENOMEM, "mge_set_geometry: device allocation failed");
        }
        ECK(hipMemcpy(e->cov, cov.data(), 8 * e->ncov, hipMemcpyHostToDevice));
    }
    e->nb = nb;
    if (nb > 0) ECK(hipMemcpy(e->bidx, bidx, 8 * nb, hipMemcpyHostToDevice));
    double *d_boff = nullptr, *pcb = nullptr;  // surface points; the preconditioner's faces and diagonal
    if ((nb > 0 && hipMalloc(&d_boff, 24 * nb) != hipSuccess) ||
        hipMalloc(&pcb, 8 * (nfx + nfy + nfz + n)) != hipSuccess) {
        if (d_boff) (void)hipFree(d_boff);
        free_geometry(e);
        return set_err(MG_ENOMEM, "mge_set_geometry: device allocation failed");
    }
    double *pbx = pcb, *pby = pcb + nfx, *pbz = pcb + nfx + nfy, *pdiag = pcb + nfx + nfy + nfz;
    if (nb > 0) ECK(hipMemcpy(d_boff, boff, 24 * nb, hipMemcpyHostToDevice));
    e->G.a = a;
    e->G.bcmask = mask;
    for (int f = 0; f < 6; ++f) e->G.g[f] = (mask >> f & 1) ? bc->value[f] : 0.0;
    e->g_eb = g_eb;
    hipLaunchKernelGGL(eb_pc_faces_k, dim3(grid1(nfx + nfy + nfz)), dim3(256), 0, s, e->ax, e->ay, e->az, e->eps,
                       e->G, pbx, pby, pbz);
    hipLaunchKernelGGL(eb_pc_diag_k, dim3(grid1(n)), dim3(256), 0, s, e->kappa, e->G, pdiag, n);
    if (nb > 0)
        hipLaunchKernelGGL(eb_setup_k, dim3(grid1(nb)), dim3(256), 0, s, e->bidx, d_boff, e->eps, e->ax, e->ay,
                           e->az, e->G, nb, e->sidx, e->sw, e->c15, pdiag);
    const hipError_t le = hipGetLastError();
    const hipError_t se = hipStreamSynchronize(s);
    if (d_boff) (void)hipFree(d_boff);
    if (le != hipSuccess || se != hipSuccess) (void)hipFree(pcb);
    ECK(le);
    ECK(se);
    // the preconditioner's operator: the symmetric part of the cut-cell
    // operator, zero box-face values (its a enters through the diagonal)
    mg_bcs hb = *bc;
    for (int f = 0; f < 6; ++f) hb.value[f] = 0.0;
    const int prc = mg_set_face_coeffs_diag(e->pc, pbx, pby, pbz, pdiag, 0.0, &hb);
    (void)hipFree(pcb);
    if (prc != MG_OK) {
        free_geometry(e);
        return prc;
    }
    e->ready = true;
    return MG_OK;
}

int mge_apply(mge_ctx *e, const double *x, double *y) {
    if (!e || !x || !y) return set_err(MG_EINVAL, "mge_apply: null argument");
    if (!e->ready) return set_err(MG_EINVAL, "mge_apply: mge_set_geometry has not succeeded");
    if (x == y) return set_err(MG_EINVAL, "mge_apply: x and y must not be the same array");
    if (int rc = apply(e, x, y)) return rc;
    ECK(hipStreamSynchronize(e->stream));
    return MG_OK;
}

int mge_rhs(mge_ctx *e, const double *f, double *b) {
    if (!e || !f || !b) return set_err(MG_EINVAL, "mge_rhs: null argument");
    if (!e->ready) return set_err(MG_EINVAL, "mge_rhs: mge_set_geometry has not succeeded");
    if (int rc = rhs(e, f, b)) return rc;
    ECK(hipStreamSynchronize(e->stream));
    return MG_OK;
}

int mge_timing(mge_ctx *e, int enable) {
    if (!e) return set_err(MG_EINVAL, "mge_timing: null context");
    return mg_timing(e->pc, enable);
}

int mge_timing_read(const mge_ctx *e, long *launches, double *ms, double *bytes, const char **kernel) {
    if (!e) return set_err(MG_EINVAL, "mge_timing_read: null context");
    return mg_timing_read(e->pc, launches, ms, bytes, kernel);
}

int mge_solve(mge_ctx *e, const double *f, double *x, unsigned flags, mg_stats *st) {
    auto t0 = std::chrono::steady_clock::now();
    if (!e || !f || !x) return set_err(MG_EINVAL, "mge_solve: null argument");
    if (!e->ready) return set_err(MG_EINVAL, "mge_solve: mge_set_geometry has not succeeded");
    if (flags & ~(unsigned)MG_GUESS) return set_err(MG_EINVAL, "mge_solve: unknown flags 0x%x", flags);
    hipStream_t s = e->stream;
    int rc;
    if ((rc = rhs(e, f, e->b))) return rc;
    if (!(flags & MG_GUESS)) ECK(fill_zero(s, x, e->n * 8));
    if (e->ncov > 0) {  // covered rows hold from the start
        hipLaunchKernelGGL(eb_set_list_k, dim3(grid1(e->ncov)), dim3(256), 0, s, x, e->cov, e->ncov, e->gc, e->g_eb);
        ECK(hipGetLastError());
    }
    mg_stats S{};
    const int res = bicgstab(
        e->K, [&](const double *u, double *y) { return apply(e, u, y); },
        [&](double *v, double *z) { return precond(e, v, z); }, e->b, x, e->d.rtol, e->d.max_cycles, S,
        "mge_solve");
    if (res < 0 && res != MG_EDIVERGED) return res;
    ECK(hipStreamSynchronize(s));
    if ((rc = timing_flush(e->pc))) return rc;
    S.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (st) *st = S;
    return res;
}

}  // extern "C"
