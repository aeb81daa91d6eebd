// Composite (two-level AMR) solves: the C ABI of mga.h.
//
// Unknowns live in one composite vector: the base cells (C order), then the
// cells of each box (C order of the box).  Covered base cells are carried
// but hold no equation: their entries stay 0 in every vector of the
// iteration, so inner products and the base-grid operator need no mask.
//
// The composite operator is the single-grid operator of the base grid (the
// engine's kernel, over every base cell) corrected at the few base cells
// beside a box (their coarse-fine faces take the refluxed fine fluxes
// instead) plus one kernel over the fine cells.  BiCGStab with a right
// preconditioner runs with its scalars on the device (one host
// synchronisation per iteration, for the convergence test); the
// preconditioner is one V-cycle of the engine on the base grid, whose
// covered cells take the mean of the fine residual below them, and one
// V-cycle per box with zero correction values on its boundary, plus the
// interpolated base correction.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "mg_engine.h"
#include "mg_krylov.h"
#include "mg_stencil.cuh"
#include "mga.h"

namespace mg {

struct AmrBox {
    int lo[3];   // first fine cell (global fine indices)
    int n[3];    // fine cells per axis
    long off;    // offset of the box in the composite vector
};

struct AmrGeo {
    int nx, ny, nz;  // base grid
    double hc, hf;
    double a;
    int bcmask;
    double g[6];
    int nbox;
    long nc, ntot;
};

constexpr int kAmrMaxBoxes = 256;
constexpr int kAmrBoxStreams = 4;  // streams for the boxes' V-cycles

namespace {

__device__ __forceinline__ double harm2(double p, double q) { return 2.0 * p * q / (p + q); }

__device__ __forceinline__ long base_idx(const AmrGeo &G, int i, int j, int k) {
    return ((long)k * G.ny + j) * G.nx + i;
}

// Value of the coarse cell C moved to a ghost's tangential position along
// the two axes other than `axis`: C + sum_t s_t (C_{+t} - C_{-t}) / 8, with
// s_t = +1 for a ghost in the upper half of C along t (odd fine index).
__device__ __forceinline__ double coarse_at_ghost(const AmrGeo &G, const double *x, const int C[3], int axis,
                                                  const int gfine[3]) {
    double v = x[base_idx(G, C[0], C[1], C[2])];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        if (t == axis) continue;
        int up[3] = {C[0], C[1], C[2]}, dn[3] = {C[0], C[1], C[2]};
        up[t] += 1;
        dn[t] -= 1;
        const double s = (gfine[t] & 1) ? 0.125 : -0.125;
        v += s * (x[base_idx(G, up[0], up[1], up[2])] - x[base_idx(G, dn[0], dn[1], dn[2])]);
    }
    return v;
}

// The box of composite index i >= nc (boxes are few: a linear search).
__device__ __forceinline__ int box_of(const AmrBox *B, int nbox, long i) {
    int p = 0;
    while (p + 1 < nbox && i >= B[p + 1].off) ++p;
    return p;
}

__device__ __forceinline__ void fine_coords(const AmrBox &bx, long l, int L[3]) {
    L[0] = (int)(l % bx.n[0]);
    L[1] = (int)((l / bx.n[0]) % bx.n[1]);
    L[2] = (int)(l / ((long)bx.n[0] * bx.n[1]));
}

__device__ __forceinline__ long fine_index(const AmrBox &bx, int f0, int f1, int f2) {
    return bx.off + ((long)(f2 - bx.lo[2]) * bx.n[1] + (f1 - bx.lo[1])) * bx.n[0] + (f0 - bx.lo[0]);
}

// Base cells beside a box (list cf): the single-grid operator applied over
// the base grid took a plain face to each covered neighbour N; replace it
// by the four fine fluxes through that face (refluxing), each with the
// ghost value of its fine cell.  x is 0 on covered cells.
__global__ __launch_bounds__(256) void amr_cf_fix_k(const double *__restrict__ x, double *__restrict__ y,
                                                    const long *__restrict__ cf, long ncf,
                                                    const int *__restrict__ mask, const AmrBox *__restrict__ B,
                                                    const double *__restrict__ eps, AmrGeo G) {
    const double ic2 = 1.0 / (G.hc * G.hc), wf = 1.0 / (8.0 * G.hf * G.hf);
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < ncf; q += (long)gridDim.x * blockDim.x) {
        const long i = cf[q];
        const int I = (int)(i % G.nx), J = (int)((i / G.nx) % G.ny), K = (int)(i / ((long)G.nx * G.ny));
        const int C[3] = {I, J, K};
        const double uC = x[i], bC = eps ? eps[i] : 1.0;
        const int dims[3] = {G.nx, G.ny, G.nz};
        double acc = 0.0;
        for (int d = 0; d < 6; ++d) {
            const int axis = d >> 1, dir = (d & 1) ? 1 : -1;
            int N[3] = {I, J, K};
            N[axis] += dir;
            if (N[axis] < 0 || N[axis] >= dims[axis]) continue;
            const long ni = base_idx(G, N[0], N[1], N[2]);
            const int p = mask[ni];
            if (p < 0) continue;
            acc -= harm2(bC, eps ? eps[ni] : 1.0) * ic2 * (uC - x[ni]);
            const AmrBox &bx = B[p];
            int f[3];
            f[axis] = 2 * N[axis] + (dir < 0 ? 1 : 0);
            const int t1 = axis == 0 ? 1 : 0, t2 = axis == 2 ? 1 : 2;
            for (int o = 0; o < 4; ++o) {
                f[t1] = 2 * C[t1] + (o & 1);
                f[t2] = 2 * C[t2] + (o >> 1);
                const long fi = fine_index(bx, f[0], f[1], f[2]);
                const double uF = x[fi];
                const double bi = harm2(eps ? eps[fi] : 1.0, bC);
                // the ghost of F beyond the face lies in C, at F's tangential position
                int gf[3] = {f[0], f[1], f[2]};
                gf[axis] -= dir;
                const double Gv = uF / 3.0 + (2.0 / 3.0) * coarse_at_ghost(G, x, C, axis, gf);
                acc += bi * wf * (Gv - uF);
            }
        }
        y[i] += acc;
    }
}

// Fine cells: y = A x with the single-grid stencil inside the box and the
// ghost value beyond each coarse-fine face; the thread of the first child
// of each covered base cell sets y there to 0.
__global__ __launch_bounds__(256) void amr_fine_apply_k(const double *__restrict__ x, double *__restrict__ y,
                                                        const AmrBox *__restrict__ B, const double *__restrict__ eps,
                                                        AmrGeo G) {
    const double if2 = 1.0 / (G.hf * G.hf);
    for (long i = G.nc + (long)blockIdx.x * blockDim.x + threadIdx.x; i < G.ntot;
         i += (long)gridDim.x * blockDim.x) {
        const AmrBox &bx = B[box_of(B, G.nbox, i)];
        int L[3];
        fine_coords(bx, i - bx.off, L);
        const double uF = x[i], bF = eps ? eps[i] : 1.0;
        double acc = G.a * uF;
        const long strides[3] = {1, bx.n[0], (long)bx.n[0] * bx.n[1]};
        for (int d = 0; d < 6; ++d) {
            const int axis = d >> 1, dir = (d & 1) ? 1 : -1;
            const int nl = L[axis] + dir;
            if (nl >= 0 && nl < bx.n[axis]) {
                const long ni = i + dir * strides[axis];
                acc += harm2(bF, eps ? eps[ni] : 1.0) * if2 * (uF - x[ni]);
                continue;
            }
            // coarse-fine face: the ghost beyond it, in the coarse cell holding it
            int gf[3] = {bx.lo[0] + L[0], bx.lo[1] + L[1], bx.lo[2] + L[2]};
            gf[axis] += dir;
            const int C[3] = {gf[0] >> 1, gf[1] >> 1, gf[2] >> 1};
            const double bi = harm2(bF, eps ? eps[base_idx(G, C[0], C[1], C[2])] : 1.0);
            const double Gv = uF / 3.0 + (2.0 / 3.0) * coarse_at_ghost(G, x, C, axis, gf);
            acc += bi * if2 * (uF - Gv);
        }
        y[i] = acc;
        if (((L[0] | L[1] | L[2]) & 1) == 0)
            y[base_idx(G, (bx.lo[0] + L[0]) >> 1, (bx.lo[1] + L[1]) >> 1, (bx.lo[2] + L[2]) >> 1)] = 0.0;
    }
}

// b = f plus the Dirichlet terms of the base cells on the domain faces; 0
// on covered base cells.  b already holds f.
__global__ void amr_rhs_k(double *__restrict__ b, const int *__restrict__ mask, const double *__restrict__ eps,
                          AmrGeo G) {
    const double ic2 = 1.0 / (G.hc * G.hc);
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < G.nc; i += (long)gridDim.x * blockDim.x) {
        if (mask[i] >= 0) {
            b[i] = 0.0;
            continue;
        }
        const int I = (int)(i % G.nx), J = (int)((i / G.nx) % G.ny), K = (int)(i / ((long)G.nx * G.ny));
        const bool at[6] = {I == 0, I == G.nx - 1, J == 0, J == G.ny - 1, K == 0, K == G.nz - 1};
        const double be = eps ? eps[i] : 1.0;
        double add = 0.0;
        for (int d = 0; d < 6; ++d)
            if (at[d] && ((G.bcmask >> d) & 1)) add += 2.0 * be * G.g[d];
        b[i] += ic2 * add;
    }
}

// Covered base cells of v: the mean of the eight fine values below them
// (one thread per covered cell; list of covered cells with their box).
__global__ void amr_restrict_k(double *__restrict__ v, const long *__restrict__ cov, const int *__restrict__ mask,
                               long ncov, const AmrBox *__restrict__ B, AmrGeo G) {
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < ncov; q += (long)gridDim.x * blockDim.x) {
        const long i = cov[q];
        const int I = (int)(i % G.nx), J = (int)((i / G.nx) % G.ny), K = (int)(i / ((long)G.nx * G.ny));
        const AmrBox &bx = B[mask[i]];
        double s = 0.0;
        for (int o = 0; o < 8; ++o)
            s += v[fine_index(bx, 2 * I + (o & 1), 2 * J + ((o >> 1) & 1), 2 * K + (o >> 2))];
        v[i] = 0.125 * s;
    }
}

__global__ void amr_zero_list_k(double *__restrict__ v, const long *__restrict__ cov, long ncov) {
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < ncov; q += (long)gridDim.x * blockDim.x)
        v[cov[q]] = 0.0;
}

// z_fine += the cell-centred trilinear interpolation of the base part of z
__global__ void amr_interp_k(double *__restrict__ z, const AmrBox *__restrict__ B, AmrGeo G) {
    for (long i = G.nc + (long)blockIdx.x * blockDim.x + threadIdx.x; i < G.ntot;
         i += (long)gridDim.x * blockDim.x) {
        const AmrBox &bx = B[box_of(B, G.nbox, i)];
        int L[3];
        fine_coords(bx, i - bx.off, L);
        const int f[3] = {bx.lo[0] + L[0], bx.lo[1] + L[1], bx.lo[2] + L[2]};
        const int C[3] = {f[0] >> 1, f[1] >> 1, f[2] >> 1};
        const int s[3] = {(f[0] & 1) ? 1 : -1, (f[1] & 1) ? 1 : -1, (f[2] & 1) ? 1 : -1};
        double v = 0.0;
        for (int o = 0; o < 8; ++o) {
            const int a = o & 1, bb = (o >> 1) & 1, c = o >> 2;
            const double w = (a ? 0.25 : 0.75) * (bb ? 0.25 : 0.75) * (c ? 0.25 : 0.75);
            v += w * z[base_idx(G, C[0] + a * s[0], C[1] + bb * s[1], C[2] + c * s[2])];
        }
        z[i] += v;
    }
}

// covered base cells of the solution: the mean of their eight children
__global__ void amr_average_down_k(double *__restrict__ xb, const double *__restrict__ x,
                                   const long *__restrict__ cov, const int *__restrict__ mask, long ncov,
                                   const AmrBox *__restrict__ B, AmrGeo G) {
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < ncov; q += (long)gridDim.x * blockDim.x) {
        const long i = cov[q];
        const int I = (int)(i % G.nx), J = (int)((i / G.nx) % G.ny), K = (int)(i / ((long)G.nx * G.ny));
        const AmrBox &bx = B[mask[i]];
        double s = 0.0;
        for (int o = 0; o < 8; ++o)
            s += x[fine_index(bx, 2 * I + (o & 1), 2 * J + ((o >> 1) & 1), 2 * K + (o >> 2))];
        xb[i] = 0.125 * s;
    }
}

__global__ void amr_fill_mask_k(int *mask, long nc) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += (long)gridDim.x * blockDim.x) mask[i] = -1;
}
__global__ void amr_mark_k(int *mask, const long *cov, const int *owner, long ncov) {
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < ncov; q += (long)gridDim.x * blockDim.x)
        mask[cov[q]] = owner[q];
}

unsigned grid1(long n) { return (unsigned)std::min<long>(std::max<long>((n + 255) / 256, 1), 16384); }

}  // namespace
}  // namespace mg

struct mga_ctx {
    mg_desc d{};
    hipStream_t stream = nullptr;
    mg::AmrGeo G{};
    std::vector<mg::AmrBox> hboxes;
    mg::AmrBox *dboxes = nullptr;
    int *mask = nullptr;
    long *cf = nullptr, *cov = nullptr;  // base cells beside a box; covered base cells
    long ncf = 0, ncov = 0;
    double *eps = nullptr;  // composite coefficient vector (or null)
    double *vec = nullptr;  // two composite vectors: x and b (b serves mga_apply's output)
    mg::KrylovSpace K;      // the iteration's vectors (covered entries stay 0) and reductions
    mg_ctx *base = nullptr;    // base-grid operator with zero boundary values
    std::vector<mg_ctx *> pc;  // one per box, zero values on its boundary
    // the boxes' V-cycles run on a few streams of their own, beside the base cycle
    std::vector<hipStream_t> ps;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> join;
    bool coeffs = false;
};

using namespace mg;

namespace {

#define ACK(expr)                                                                                  \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return set_err(MG_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),       \
                           __FILE__, __LINE__);                                                    \
    } while (0)

enum { V_X = 0, V_B, V_NUM };

double *vecp(mga_ctx *m, int k) { return m->vec + (size_t)k * m->G.ntot; }

// y = A x (x zero on covered cells; y zero there afterwards)
int apply(mga_ctx *m, const double *x, double *y) {
    hipStream_t s = m->stream;
    ACK(apply_op(s, level_geo(m->base, 0, false), level_coef(m->base, 0, false), 0.0, 1.0, x, y));
    if (m->ncf > 0)
        hipLaunchKernelGGL(amr_cf_fix_k, dim3(grid1(m->ncf)), dim3(256), 0, s, x, y, m->cf, m->ncf, m->mask,
                           m->dboxes, m->eps, m->G);
    ACK(hipGetLastError());
    if (m->G.ntot > m->G.nc)
        hipLaunchKernelGGL(amr_fine_apply_k, dim3(grid1(m->G.ntot - m->G.nc)), dim3(256), 0, s, x, y, m->dboxes,
                           m->eps, m->G);
    ACK(hipGetLastError());
    return MG_OK;
}

// One V-cycle of context c from zero on b, into x (no synchronisation).
int vcycle_once(mg_ctx *c, const double *b, double *x) {
    std::vector<LvView> V;
    fp64_view(c, V, b, x);
    if (int rc = vcycle(c, V, 0, true)) return rc;
    if (V[0].u != x) ACK(hipMemcpyAsync(x, V[0].u, c->L[0].n * 8, hipMemcpyDeviceToDevice, c->stream));
    return MG_OK;
}

// z = M^-1 v.  v's covered entries hold the restricted fine part while the
// base cycle runs and are 0 again afterwards.
int precond(mga_ctx *m, double *v, double *z) {
    hipStream_t s = m->stream;
    if (m->ncov > 0) {
        hipLaunchKernelGGL(amr_restrict_k, dim3(grid1(m->ncov)), dim3(256), 0, s, v, m->cov, m->mask, m->ncov,
                           m->dboxes, m->G);
        ACK(hipGetLastError());
    }
    // fork: the boxes' cycles start once the restriction is enqueued (they
    // read v's fine part, the base cycle its base part; they write disjoint
    // parts of z)
    const int K = (int)m->ps.size();
    if (K > 0) {
        ACK(hipEventRecord(m->fork, s));
        for (int q = 0; q < K; ++q) ACK(hipStreamWaitEvent(m->ps[q], m->fork, 0));
    }
    for (int p = 0; p < m->G.nbox; ++p) {
        const long off = m->hboxes[p].off;
        if (int rc = vcycle_once(m->pc[p], v + off, z + off)) return rc;
    }
    for (int q = 0; q < K; ++q) ACK(hipEventRecord(m->join[q], m->ps[q]));
    if (int rc = vcycle_once(m->base, v, z)) return rc;
    for (int q = 0; q < K; ++q) ACK(hipStreamWaitEvent(s, m->join[q], 0));
    if (m->ncov > 0) {
        hipLaunchKernelGGL(amr_interp_k, dim3(grid1(m->G.ntot - m->G.nc)), dim3(256), 0, s, z, m->dboxes, m->G);
        hipLaunchKernelGGL(amr_zero_list_k, dim3(grid1(m->ncov)), dim3(256), 0, s, z, m->cov, m->ncov);
        hipLaunchKernelGGL(amr_zero_list_k, dim3(grid1(m->ncov)), dim3(256), 0, s, v, m->cov, m->ncov);
        ACK(hipGetLastError());
    }
    return MG_OK;
}

// copy the caller's base + box arrays into a composite vector
int pack(mga_ctx *m, double *dst, const double *base, const double *const *fine) {
    ACK(hipMemcpyAsync(dst, base, m->G.nc * 8, hipMemcpyDeviceToDevice, m->stream));
    for (int p = 0; p < m->G.nbox; ++p) {
        const AmrBox &b = m->hboxes[p];
        ACK(hipMemcpyAsync(dst + b.off, fine[p], (size_t)b.n[0] * b.n[1] * b.n[2] * 8, hipMemcpyDeviceToDevice,
                           m->stream));
    }
    return MG_OK;
}

int zero_covered(mga_ctx *m, double *v) {
    if (m->ncov > 0) {
        hipLaunchKernelGGL(amr_zero_list_k, dim3(grid1(m->ncov)), dim3(256), 0, m->stream, v, m->cov, m->ncov);
        ACK(hipGetLastError());
    }
    return MG_OK;
}

int unpack(mga_ctx *m, const double *src, double *base, double *const *fine, bool average_down) {
    ACK(hipMemcpyAsync(base, src, m->G.nc * 8, hipMemcpyDeviceToDevice, m->stream));
    if (average_down && m->ncov > 0)
        hipLaunchKernelGGL(amr_average_down_k, dim3(grid1(m->ncov)), dim3(256), 0, m->stream, base, src, m->cov,
                           m->mask, m->ncov, m->dboxes, m->G);
    ACK(hipGetLastError());
    for (int p = 0; p < m->G.nbox; ++p) {
        const AmrBox &b = m->hboxes[p];
        ACK(hipMemcpyAsync(fine[p], src + b.off, (size_t)b.n[0] * b.n[1] * b.n[2] * 8, hipMemcpyDeviceToDevice,
                           m->stream));
    }
    return MG_OK;
}

bool boxes_ok(const mg_desc *d, int nbox, const mga_box *bx, char *why, size_t nwhy) {
    const int dims[3] = {d->nx, d->ny, d->nz};
    for (int p = 0; p < nbox; ++p)
        for (int a = 0; a < 3; ++a) {
            const int lo = bx[p].lo[a], hi = bx[p].hi[a];
            if ((lo & 1) || (hi & 1) || hi <= lo) {
                snprintf(why, nwhy, "box %d: bounds must be even with hi > lo", p);
                return false;
            }
            if (lo < 2 || hi > 2 * dims[a] - 2) {
                snprintf(why, nwhy, "box %d must stay one coarse cell inside the domain", p);
                return false;
            }
        }
    for (int p = 0; p < nbox; ++p)
        for (int q = p + 1; q < nbox; ++q) {
            bool close = true;
            for (int a = 0; a < 3; ++a)
                close = close && bx[p].lo[a] - 2 < bx[q].hi[a] && bx[q].lo[a] < bx[p].hi[a] + 2;
            if (close) {
                snprintf(why, nwhy, "boxes %d and %d are less than one coarse cell apart", p, q);
                return false;
            }
        }
    return true;
}

// Covered base cells (with their box) and the uncovered base cells beside
// a box face, sorted, on the host.
void cell_lists(const mg_desc *d, int nbox, const mga_box *bx, std::vector<long> &cov, std::vector<int> &owner,
                std::vector<long> &cf) {
    const long nx = d->nx, ny = d->ny;
    auto idx = [&](long i, long j, long k) { return (k * ny + j) * nx + i; };
    for (int p = 0; p < nbox; ++p) {
        int L[3], H[3];
        for (int a = 0; a < 3; ++a) {
            L[a] = bx[p].lo[a] / 2;
            H[a] = bx[p].hi[a] / 2;
        }
        for (int k = L[2]; k < H[2]; ++k)
            for (int j = L[1]; j < H[1]; ++j)
                for (int i = L[0]; i < H[0]; ++i) {
                    cov.push_back(idx(i, j, k));
                    owner.push_back(p);
                }
        for (int a = 0; a < 3; ++a)
            for (int side = 0; side < 2; ++side) {
                int lo[3] = {L[0], L[1], L[2]}, hi[3] = {H[0], H[1], H[2]};
                lo[a] = side ? H[a] : L[a] - 1;
                hi[a] = lo[a] + 1;
                for (int k = lo[2]; k < hi[2]; ++k)
                    for (int j = lo[1]; j < hi[1]; ++j)
                        for (int i = lo[0]; i < hi[0]; ++i) cf.push_back(idx(i, j, k));
            }
    }
    std::sort(cf.begin(), cf.end());
    cf.erase(std::unique(cf.begin(), cf.end()), cf.end());
}

}  // namespace

extern "C" {

int mga_destroy(mga_ctx *m) {
    if (!m) return MG_OK;
    (void)hipStreamSynchronize(m->stream);
    for (hipStream_t q : m->ps) (void)hipStreamSynchronize(q);
    if (m->base) mg_destroy(m->base);
    for (mg_ctx *c : m->pc) mg_destroy(c);
    for (hipStream_t q : m->ps) (void)hipStreamDestroy(q);
    for (hipEvent_t e : m->join) (void)hipEventDestroy(e);
    if (m->fork) (void)hipEventDestroy(m->fork);
    for (void *p : {(void *)m->dboxes, (void *)m->mask, (void *)m->cf, (void *)m->cov, (void *)m->eps,
                    (void *)m->vec})
        if (p) (void)hipFree(p);
    krylov_free(m->K);
    delete m;
    return MG_OK;
}

int mga_create(const mg_desc *d, int nbox, const mga_box *boxes, void *hip_stream, mga_ctx **out) {
    if (out) *out = nullptr;
    if (!d || !out || nbox < 0 || (nbox > 0 && !boxes)) return set_err(MG_EINVAL, "mga_create: bad argument");
    if (nbox > kAmrMaxBoxes) return set_err(MG_EINVAL, "mga_create: at most %d boxes", kAmrMaxBoxes);
    if (d->precision != MG_FP64) return set_err(MG_EINVAL, "mga_create: composite solves run in MG_FP64");
    if (int rc = check_grid("mga_create", d)) return rc;
    char why[160];
    if (!boxes_ok(d, nbox, boxes, why, sizeof why)) return set_err(MG_EINVAL, "mga_create: %s", why);
    mga_ctx *m = new mga_ctx();
    m->d = *d;
    m->stream = (hipStream_t)hip_stream;
    AmrGeo &G = m->G;
    G.nx = d->nx;
    G.ny = d->ny;
    G.nz = d->nz;
    G.hc = d->h;
    G.hf = 0.5 * d->h;
    G.nbox = nbox;
    G.nc = (long)d->nx * d->ny * d->nz;
    long off = G.nc;
    for (int p = 0; p < nbox; ++p) {
        AmrBox b{};
        for (int a = 0; a < 3; ++a) {
            b.lo[a] = boxes[p].lo[a];
            b.n[a] = boxes[p].hi[a] - boxes[p].lo[a];
        }
        b.off = off;
        off += (long)b.n[0] * b.n[1] * b.n[2];
        m->hboxes.push_back(b);
    }
    G.ntot = off;
    // preconditioner contexts (their V-cycles run directly, one per call)
    int rc = mg_create(d, hip_stream, &m->base);
    const int K = std::min(nbox, kAmrBoxStreams);
    for (int q = 0; q < K && rc == MG_OK; ++q) {
        hipStream_t st = nullptr;
        hipEvent_t ev = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            rc = set_err(MG_EDEVICE, "mga_create: stream creation failed");
            break;
        }
        m->ps.push_back(st);
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            rc = set_err(MG_EDEVICE, "mga_create: event creation failed");
            break;
        }
        m->join.push_back(ev);
    }
    if (rc == MG_OK && K > 0 && hipEventCreateWithFlags(&m->fork, hipEventDisableTiming) != hipSuccess)
        rc = set_err(MG_EDEVICE, "mga_create: event creation failed");
    for (int p = 0; p < nbox && rc == MG_OK; ++p) {
        mg_desc pd = *d;
        pd.nx = m->hboxes[p].n[0];
        pd.ny = m->hboxes[p].n[1];
        pd.nz = m->hboxes[p].n[2];
        pd.h = G.hf;
        mg_ctx *c = nullptr;
        rc = mg_create(&pd, m->ps[p % K], &c);
        if (rc == MG_OK) m->pc.push_back(c);
        else set_err(rc, "mga_create: box %d cannot be coarsened to a bottom grid (%s)", p, mg_last_error());
    }
    if (rc != MG_OK) {
        mga_destroy(m);
        return rc;
    }
    std::vector<long> cov, cf;
    std::vector<int> owner;
    cell_lists(d, nbox, boxes, cov, owner, cf);
    m->ncov = (long)cov.size();
    m->ncf = (long)cf.size();
    int *d_owner = nullptr;
    bool ok = hipMalloc(&m->dboxes, sizeof(AmrBox) * std::max(1, nbox)) == hipSuccess &&
              hipMalloc(&m->mask, sizeof(int) * G.nc) == hipSuccess &&
              hipMalloc(&m->cov, sizeof(long) * std::max<long>(1, m->ncov)) == hipSuccess &&
              hipMalloc(&d_owner, sizeof(int) * std::max<long>(1, m->ncov)) == hipSuccess &&
              hipMalloc(&m->cf, sizeof(long) * std::max<long>(1, m->ncf)) == hipSuccess &&
              hipMalloc(&m->vec, sizeof(double) * V_NUM * G.ntot) == hipSuccess;
    if (!ok) {
        if (d_owner) (void)hipFree(d_owner);
        mga_destroy(m);
        return set_err(MG_ENOMEM, "mga_create: device allocation failed");
    }
    hipStream_t s = m->stream;
    bool cp = true;
    if (nbox > 0)
        cp = hipMemcpyAsync(m->dboxes, m->hboxes.data(), sizeof(AmrBox) * nbox, hipMemcpyHostToDevice, s) ==
                 hipSuccess &&
             hipMemcpyAsync(m->cov, cov.data(), sizeof(long) * m->ncov, hipMemcpyHostToDevice, s) == hipSuccess &&
             hipMemcpyAsync(d_owner, owner.data(), sizeof(int) * m->ncov, hipMemcpyHostToDevice, s) == hipSuccess &&
             hipMemcpyAsync(m->cf, cf.data(), sizeof(long) * m->ncf, hipMemcpyHostToDevice, s) == hipSuccess;
    hipLaunchKernelGGL(amr_fill_mask_k, dim3(grid1(G.nc)), dim3(256), 0, s, m->mask, G.nc);
    if (m->ncov > 0) hipLaunchKernelGGL(amr_mark_k, dim3(grid1(m->ncov)), dim3(256), 0, s, m->mask, m->cov, d_owner,
                                        m->ncov);
    // zero the vectors once: covered entries stay 0 from here on
    cp = cp && fill_zero(s, m->vec, sizeof(double) * V_NUM * G.ntot) == hipSuccess;
    cp = cp && hipStreamSynchronize(s) == hipSuccess;
    (void)hipFree(d_owner);
    if (!cp) {
        mga_destroy(m);
        return set_err(MG_EDEVICE, "mga_create: set-up copies or kernels failed");
    }
    // inner products weigh a base cell 8 fine cells (covered entries are 0)
    if ((rc = krylov_alloc(m->K, s, G.ntot, G.nc, 8.0))) {
        mga_destroy(m);
        return rc;
    }
    *out = m;
    return MG_OK;
}

int mga_set_coeffs(mga_ctx *m, const double *eps_base, const double *const *eps_fine, double a, const mg_bcs *bc) {
    if (!m || !bc) return set_err(MG_EINVAL, "mga_set_coeffs: null argument");
    if ((eps_base == nullptr) != (eps_fine == nullptr))
        return set_err(MG_EINVAL, "mga_set_coeffs: give both eps_base and eps_fine, or neither");
    for (int p = 0; eps_fine && p < m->G.nbox; ++p)
        if (!eps_fine[p]) return set_err(MG_EINVAL, "mga_set_coeffs: eps_fine[%d] is null", p);
    int mask = 0;
    if (int rc = parse_operator("mga_set_coeffs", a, bc, &mask)) return rc;
    m->coeffs = false;
    hipStream_t s = m->stream;
    if (eps_base) {
        if (!m->eps && hipMalloc(&m->eps, sizeof(double) * m->G.ntot) != hipSuccess)
            return set_err(MG_ENOMEM, "mga_set_coeffs: allocation failed");
        if (int rc = pack(m, m->eps, eps_base, eps_fine)) return rc;
        ACK(count_bad(s, m->eps, m->G.ntot, m->K.ws, 0));
        ACK(hipMemcpyAsync(m->K.h_pin, m->K.ws.result, sizeof(double), hipMemcpyDeviceToHost, s));
        ACK(hipStreamSynchronize(s));
        if (m->K.h_pin[0] != 0.0)
            return set_err(MG_EINVAL, "mga_set_coeffs: %.0f coefficient entries are not in (0, 1e100]",
                           m->K.h_pin[0]);
    } else if (m->eps) {
        (void)hipFree(m->eps);
        m->eps = nullptr;
    }
    // the base operator (all base cells) and the boxes' operators, zero boundary values
    mg_bcs hb = *bc;
    for (int f = 0; f < 6; ++f) hb.value[f] = 0.0;
    if (int rc = mg_set_coeffs(m->base, eps_base, a, &hb)) return rc;
    mg_bcs pb{};
    for (int f = 0; f < 6; ++f) pb.type[f] = MG_BC_DIRICHLET;
    // the boxes' streams read the caller's arrays after the work enqueued so far
    if (!m->ps.empty()) {
        ACK(hipEventRecord(m->fork, s));
        for (hipStream_t q : m->ps) ACK(hipStreamWaitEvent(q, m->fork, 0));
    }
    for (int p = 0; p < m->G.nbox; ++p)
        if (int rc = mg_set_coeffs(m->pc[p], eps_fine ? eps_fine[p] : nullptr, a, &pb)) return rc;
    m->G.a = a;
    m->G.bcmask = mask;
    for (int f = 0; f < 6; ++f) m->G.g[f] = (mask >> f & 1) ? bc->value[f] : 0.0;
    m->coeffs = true;
    return MG_OK;
}

int mga_timing(mga_ctx *m, int enable) {
    if (!m) return set_err(MG_EINVAL, "mga_timing: null context");
    return mg_timing(m->base, enable);
}

int mga_timing_read(const mga_ctx *m, long *launches, double *ms, double *bytes, const char **kernel) {
    if (!m) return set_err(MG_EINVAL, "mga_timing_read: null context");
    return mg_timing_read(m->base, launches, ms, bytes, kernel);
}

int mga_apply(mga_ctx *m, const double *x_base, const double *const *x_fine, double *y_base, double *const *y_fine) {
    if (!m || !x_base || !y_base || (m->G.nbox > 0 && (!x_fine || !y_fine)))
        return set_err(MG_EINVAL, "mga_apply: null argument");
    if (!m->coeffs) return set_err(MG_EINVAL, "mga_apply: mga_set_coeffs has not succeeded");
    double *x = vecp(m, V_X), *y = vecp(m, V_B);
    int rc;
    if ((rc = pack(m, x, x_base, x_fine)) || (rc = zero_covered(m, x)) || (rc = apply(m, x, y)) ||
        (rc = unpack(m, y, y_base, y_fine, false)))
        return rc;
    // leave the work vectors as the solver expects them (covered entries 0)
    if ((rc = zero_covered(m, x))) return rc;
    ACK(hipStreamSynchronize(m->stream));
    return MG_OK;
}

int mga_solve(mga_ctx *m, const double *f_base, const double *const *f_fine, double *x_base, double *const *x_fine,
              unsigned flags, mg_stats *st) {
    auto t0 = std::chrono::steady_clock::now();
    if (!m || !f_base || !x_base || (m->G.nbox > 0 && (!f_fine || !x_fine)))
        return set_err(MG_EINVAL, "mga_solve: null argument");
    if (!m->coeffs) return set_err(MG_EINVAL, "mga_solve: mga_set_coeffs has not succeeded");
    if (flags & ~(unsigned)MG_GUESS) return set_err(MG_EINVAL, "mga_solve: unknown flags 0x%x", flags);
    hipStream_t s = m->stream;
    const long n = m->G.ntot;
    double *x = vecp(m, V_X), *b = vecp(m, V_B);
    int rc;
    if ((rc = pack(m, b, f_base, f_fine))) return rc;
    hipLaunchKernelGGL(amr_rhs_k, dim3(grid1(m->G.nc)), dim3(256), 0, s, b, m->mask, m->eps, m->G);
    ACK(hipGetLastError());
    if (flags & MG_GUESS) {
        if ((rc = pack(m, x, x_base, x_fine)) || (rc = zero_covered(m, x))) return rc;
    } else {
        ACK(fill_zero(s, x, n * 8));
    }
    mg_stats S{};
    const int res = bicgstab(
        m->K, [&](const double *u, double *y) { return apply(m, u, y); },
        [&](double *v, double *z) { return precond(m, v, z); }, b, x, m->d.rtol, m->d.max_cycles, S, "mga_solve");
    if (res < 0 && res != MG_EDIVERGED) return res;
    if ((rc = unpack(m, x, x_base, x_fine, true))) return rc;
    ACK(hipStreamSynchronize(s));
    if ((rc = timing_flush(m->base))) return rc;
    S.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (st) *st = S;
    return res;
}

}  // extern "C"
