// Bottom solver: one workgroup, all levels in LDS, FP64.
//
// The levels whose largest dimension is at most bottom_max (<= 16^3 cells)
// are too small to fill the GPU, so one workgroup of 1024 threads keeps
// their iterates and right-hand sides in LDS and runs the remaining part of
// the V-cycle there: red-black Gauss-Seidel smoothing, residual
// restriction, trilinear prolongation, and conjugate gradients on the
// coarsest grid (the operator is symmetric positive definite).  The paper
// pairs its red-black Gauss-Seidel multigrid with a Krylov bottom solver
// (BiCGStab); CG is the Krylov method for the SPD case.
#include "mg_stencil.cuh"

namespace mg {

namespace {

constexpr int kNT = 1024;

// off/dg of cell (i,j,k) at tail level l with operand array v (LDS).
__device__ __forceinline__ void tail_terms(const TailDesc &D, int l, const double *lds,
                                           const double *v, int i, int j, int k, bool with_g,
                                           double &off, double &dg) {
    const TailLevel &L = D.L[l];
    Geo G;
    G.nx = L.nx;
    G.ny = L.ny;
    G.nz = L.nz;
    G.bcmask = D.bcmask;
#pragma unroll
    for (int d = 0; d < 6; ++d) G.g[d] = with_g ? D.g[d] : 0.0;
    const int sy = L.nx, sz = L.nx * L.ny;
    const int p = k * sz + j * sy + i;
    // neighbours across the box boundary read the cell itself (a valid
    // address; six_faces does not use the value), so all six LDS reads are
    // issued together instead of one at a time under per-face branches
    auto un = [&](int d) -> double {
        switch (d) {
            case 0: return v[i > 0 ? p - 1 : p];
            case 1: return v[i < L.nx - 1 ? p + 1 : p];
            case 2: return v[j > 0 ? p - sy : p];
            case 3: return v[j < L.ny - 1 ? p + sy : p];
            case 4: return v[k > 0 ? p - sz : p];
            default: return v[k < L.nz - 1 ? p + sz : p];
        }
    };
    auto en = [&](int) { return 1.0; };
    if (D.mode == COEF_FACE || D.mode == COEF_FACED) {
        // face coefficients staged in LDS at the start of the kernel (or in memory)
        const double *fx = D.stage ? lds + L.off_fx : L.bx;
        const double *fy = D.stage ? lds + L.off_fy : L.by;
        const double *fz = D.stage ? lds + L.off_fz : L.bz;
        auto fb = [&](int d) -> double {
            switch (d) {
                case 0: return face_x(fx, G, i, j, k);
                case 1: return face_x(fx, G, i + 1, j, k);
                case 2: return face_y(fy, G, i, j, k);
                case 3: return face_y(fy, G, i, j + 1, k);
                case 4: return face_z(fz, G, i, j, k);
                default: return face_z(fz, G, i, j, k + 1);
            }
        };
        six_faces<double, COEF_FACE, true>(G, i, j, k, 1.0, un, en, fb, off, dg);
        if (D.mode == COEF_FACED) dg = fma(L.h2, L.dd[p], dg);  // the extra diagonal, in h^2 units
    } else {
        six_faces<double, COEF_CONST, true>(G, i, j, k, 1.0, un, en, [&](int) { return 1.0; }, off, dg);
    }
}

__device__ __forceinline__ void decode(int idx, int nx, int ny, int &i, int &j, int &k) {
    i = idx % nx;
    const int r = idx / nx;
    j = r % ny;
    k = r / ny;
}

__device__ double block_sum(double v, double *red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < kNT / 64; ++q) t += red[q];
    return t;
}

// One red-black sweep.  The threads enumerate only the cells of the colour
// being updated: item t = (h, j, k) names the h-th cell of that colour in row
// (j, k), at i = 2h + ((colour + j + k) & 1), so no lane idles on a cell of
// the other colour.  Cells of one colour are independent; the update of each
// is the same expression as for any other order.
__device__ void gs_sweep(const TailDesc &D, int l, double *lds, bool with_g) {
    const TailLevel &L = D.L[l];
    double *u = lds + L.off_u;
    const double *b = lds + L.off_b;
    const int hx = (L.nx + 1) >> 1;  // cells of one colour per row, at most
    const int m = hx * L.ny * L.nz;
    for (int colour = 0; colour < 2; ++colour) {
        for (int t = threadIdx.x; t < m; t += kNT) {
            int h, j, k;
            decode(t, hx, L.ny, h, j, k);
            const int i = 2 * h + ((colour + j + k) & 1);
            if (i >= L.nx) continue;  // odd nx: this row has one cell fewer of this colour
            const int idx = (k * L.ny + j) * L.nx + i;
            double off, dg;
            tail_terms(D, l, lds, u, i, j, k, with_g, off, dg);
            u[idx] = (L.h2 * b[idx] + off) / (L.ah2 + dg);
        }
        __syncthreads();
    }
}

__device__ __forceinline__ double tail_resid(const TailDesc &D, int l, const double *lds,
                                             const double *u, const double *b, int idx,
                                             bool with_g) {
    const TailLevel &L = D.L[l];
    int i, j, k;
    decode(idx, L.nx, L.ny, i, j, k);
    double off, dg;
    tail_terms(D, l, lds, u, i, j, k, with_g, off, dg);
    return b[idx] - (L.ah2 * u[idx] + dg * u[idx] - off) / L.h2;
}

// Restriction: the mean of the 8 children's residuals.  Thread item t is
// child t & 7 of coarse cell t >> 3, so all threads work (8 children per
// coarse cell over up to 512 coarse cells); the 8 residuals of a coarse
// cell lie in 8 adjacent lanes and are summed by lane shuffles in a fixed
// tree order.
__device__ void restrict_to(const TailDesc &D, int l, double *lds, bool with_g) {
    const TailLevel &F = D.L[l], &Cc = D.L[l + 1];
    const double *u = lds + F.off_u, *b = lds + F.off_b;
    double *bc = lds + Cc.off_b, *uc = lds + Cc.off_u;
    const int nc = Cc.nx * Cc.ny * Cc.nz;  // <= 512
    const int items = (nc * 8 + 63) / 64 * 64;  // whole waves: every lane of a group of 8 takes part
    for (int t = threadIdx.x; t < items; t += kNT) {
        const int I = t >> 3, c = t & 7;
        double s = 0.0;
        if (I < nc) {
            int ci, cj, ck;
            decode(I, Cc.nx, Cc.ny, ci, cj, ck);
            const int dx = c & 1, dy = (c >> 1) & 1, dz = c >> 2;
            const int idx = ((2 * ck + dz) * F.ny + (2 * cj + dy)) * F.nx + (2 * ci + dx);
            s = tail_resid(D, l, lds, u, b, idx, with_g);
        }
        s += __shfl_xor(s, 1, 64);
        s += __shfl_xor(s, 2, 64);
        s += __shfl_xor(s, 4, 64);
        if (I < nc && c == 0) {
            bc[I] = 0.125 * s;
            uc[I] = 0.0;
        }
    }
    __syncthreads();
}

__device__ void prolong_into(const TailDesc &D, int l, double *lds) {
    const TailLevel &F = D.L[l], &Cc = D.L[l + 1];
    double *u = lds + F.off_u;
    const double *e = lds + Cc.off_u;
    const int n = F.nx * F.ny * F.nz;
    const int m = D.bcmask;
    for (int idx = threadIdx.x; idx < n; idx += kNT) {
        int i, j, k;
        decode(idx, F.nx, F.ny, i, j, k);
        const int I = i >> 1, J = j >> 1, K = k >> 1;
        const int si = (i & 1) ? 1 : -1, sj = (j & 1) ? 1 : -1, sk = (k & 1) ? 1 : -1;
        double v = 0.0;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int bb = 0; bb < 2; ++bb)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    int ii = I + a * si, jj = J + bb * sj, kk = K + c * sk;
                    double sg = 1.0;
                    if (ii < 0) { ii = 0; if (m & 1) sg = -sg; }
                    if (ii >= Cc.nx) { ii = Cc.nx - 1; if (m & 2) sg = -sg; }
                    if (jj < 0) { jj = 0; if (m & 4) sg = -sg; }
                    if (jj >= Cc.ny) { jj = Cc.ny - 1; if (m & 8) sg = -sg; }
                    if (kk < 0) { kk = 0; if (m & 16) sg = -sg; }
                    if (kk >= Cc.nz) { kk = Cc.nz - 1; if (m & 32) sg = -sg; }
                    const double w = (a ? 0.25 : 0.75) * (bb ? 0.25 : 0.75) * (c ? 0.25 : 0.75);
                    v += w * sg * e[(kk * Cc.ny + jj) * Cc.nx + ii];
                }
        u[idx] += v;
    }
    __syncthreads();
}

// CG on level l: x = u_l (start), b_l is overwritten by the residual.
__device__ void cg_solve(const TailDesc &D, int l, double *lds, double *red, bool with_g) {
    const TailLevel &L = D.L[l];
    double *x = lds + L.off_u;
    double *r = lds + L.off_b;
    double *p = lds + D.off_p;
    double *q = lds + D.off_q;
    const int n = L.nx * L.ny * L.nz;
    // r = b - A x (boundary values only on the top level), p = r
    for (int idx = threadIdx.x; idx < n; idx += kNT) q[idx] = tail_resid(D, l, lds, x, r, idx, with_g);
    __syncthreads();
    double s = 0.0;
    for (int idx = threadIdx.x; idx < n; idx += kNT) {
        r[idx] = q[idx];
        p[idx] = q[idx];
        s += q[idx] * q[idx];
    }
    double rr = block_sum(s, red);
    const double stop = D.cg_rtol * D.cg_rtol * rr;
    for (int it = 0; it < D.cg_maxit && rr > stop && rr > 0.0; ++it) {
        double pq = 0.0;
        for (int idx = threadIdx.x; idx < n; idx += kNT) {
            int i, j, k;
            decode(idx, L.nx, L.ny, i, j, k);
            double off, dg;
            tail_terms(D, l, lds, p, i, j, k, false, off, dg);
            const double ap = (L.ah2 * p[idx] + dg * p[idx] - off) / L.h2;
            q[idx] = ap;
            pq += p[idx] * ap;
        }
        pq = block_sum(pq, red);
        const double alpha = rr / pq;
        double s2 = 0.0;
        for (int idx = threadIdx.x; idx < n; idx += kNT) {
            x[idx] += alpha * p[idx];
            r[idx] -= alpha * q[idx];
            s2 += r[idx] * r[idx];
        }
        const double rr_new = block_sum(s2, red);
        const double beta = rr_new / rr;
        rr = rr_new;
        for (int idx = threadIdx.x; idx < n; idx += kNT) p[idx] = r[idx] + beta * p[idx];
        __syncthreads();
    }
}

}  // namespace

// Bottom solve of one problem by the calling workgroup (kNT threads).
template <class T>
__device__ void tail_body(const TailDesc &D, const T *__restrict__ b_in, const T *u_in, T *u_out,
                          int top_has_g, double *lds, double *red) {
    // u_in may alias u_out: every read of u_in precedes the barrier that
    // precedes the first write of u_out.
    const TailLevel &L0 = D.L[0];
    const int n0 = L0.nx * L0.ny * L0.nz;
    if ((D.mode == COEF_FACE || D.mode == COEF_FACED) && D.stage) {
        for (int l = 0; l < D.nlev; ++l) {
            const TailLevel &L = D.L[l];
            const int nfx = (L.nx + 1) * L.ny * L.nz, nfy = L.nx * (L.ny + 1) * L.nz,
                      nfz = L.nx * L.ny * (L.nz + 1);
            for (int q = threadIdx.x; q < nfx; q += kNT) lds[L.off_fx + q] = L.bx[q];
            for (int q = threadIdx.x; q < nfy; q += kNT) lds[L.off_fy + q] = L.by[q];
            for (int q = threadIdx.x; q < nfz; q += kNT) lds[L.off_fz + q] = L.bz[q];
        }
    }
    for (int idx = threadIdx.x; idx < n0; idx += kNT) {
        lds[L0.off_b + idx] = (double)Num<T>::ld(b_in[idx]);
        lds[L0.off_u + idx] = u_in ? (double)Num<T>::ld(u_in[idx]) : 0.0;
    }
    __syncthreads();
    const int c = D.nlev - 1;
    if (c == 0) {
        cg_solve(D, 0, lds, red, top_has_g != 0);
    } else {
        for (int cyc = 0; cyc < D.ncyc; ++cyc) {
            for (int l = 0; l < c; ++l) {
                const bool g = (l == 0) && top_has_g;
                for (int s = 0; s < D.nu1; ++s) gs_sweep(D, l, lds, g);
                restrict_to(D, l, lds, g);
            }
            cg_solve(D, c, lds, red, false);
            __syncthreads();
            for (int l = c - 1; l >= 0; --l) {
                const bool g = (l == 0) && top_has_g;
                prolong_into(D, l, lds);
                for (int s = 0; s < D.nu2; ++s) gs_sweep(D, l, lds, g);
            }
        }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < n0; idx += kNT)
        u_out[idx] = Num<T>::cv(typename Num<T>::C(lds[L0.off_u + idx]));
}

template <class T>
__global__ __launch_bounds__(kNT) void tail_k(TailDesc D, const T *__restrict__ b_in, const T *u_in,
                                              T *u_out, int top_has_g, const int *__restrict__ done) {
    if (done && *done) return;
    __shared__ double lds[kTailLdsDoubles];
    __shared__ double red[kNT / 64];
    tail_body<T>(D, b_in, u_in, u_out, top_has_g, lds, red);
}

// Batched bottom solves: workgroup w solves problem w (descriptors and
// arrays per problem, problems that have converged are skipped).
template <class T>
__global__ __launch_bounds__(kNT) void tail_batched_k(const TailDesc *__restrict__ descs,
                                                      const TailIo *__restrict__ io) {
    const TailIo &q = io[blockIdx.x];
    if (q.done && *q.done) return;
    __shared__ double lds[kTailLdsDoubles];
    __shared__ double red[kNT / 64];
    tail_body<T>(descs[blockIdx.x], static_cast<const T *>(q.b), nullptr, static_cast<T *>(q.u), 0, lds, red);
}

hipError_t tail_solve_batched(hipStream_t s, int st, const TailDesc *descs, const TailIo *io, int count) {
    if (count <= 0) return hipSuccess;
    switch (st) {
        case ST_F64: hipLaunchKernelGGL(tail_batched_k<double>, dim3(count), dim3(kNT), 0, s, descs, io); break;
        case ST_F32: hipLaunchKernelGGL(tail_batched_k<float>, dim3(count), dim3(kNT), 0, s, descs, io); break;
        case ST_BF16: hipLaunchKernelGGL(tail_batched_k<bf16>, dim3(count), dim3(kNT), 0, s, descs, io); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

bool tail_layout(TailDesc &D) {
    int off = 0;
    for (int l = 0; l < D.nlev; ++l) {
        const int n = D.L[l].nx * D.L[l].ny * D.L[l].nz;
        D.L[l].off_u = off;
        off += n;
        D.L[l].off_b = off;
        off += n;
    }
    const TailLevel &C = D.L[D.nlev - 1];
    const int nc = C.nx * C.ny * C.nz;
    D.off_p = off;
    off += nc;
    D.off_q = off;
    off += nc;
    for (int l = 0; l < D.nlev; ++l) {
        TailLevel &L = D.L[l];
        L.off_fx = L.off_fy = L.off_fz = 0;
        if ((D.mode != COEF_FACE && D.mode != COEF_FACED) || !D.stage) continue;
        L.off_fx = off;
        off += (L.nx + 1) * L.ny * L.nz;
        L.off_fy = off;
        off += L.nx * (L.ny + 1) * L.nz;
        L.off_fz = off;
        off += L.nx * L.ny * (L.nz + 1);
    }
    return off <= kTailLdsDoubles;
}

hipError_t tail_solve(hipStream_t s, int st, const TailDesc &D, const void *b_in, const void *u_in,
                      void *u_out, const int *done) {
    const int has_g = (D.g[0] != 0.0 || D.g[1] != 0.0 || D.g[2] != 0.0 || D.g[3] != 0.0 ||
                       D.g[4] != 0.0 || D.g[5] != 0.0);
    switch (st) {
        case ST_F64:
            hipLaunchKernelGGL(tail_k<double>, dim3(1), dim3(kNT), 0, s, D, (const double *)b_in,
                               (const double *)u_in, (double *)u_out, has_g, done);
            break;
        case ST_F32:
            hipLaunchKernelGGL(tail_k<float>, dim3(1), dim3(kNT), 0, s, D, (const float *)b_in,
                               (const float *)u_in, (float *)u_out, has_g, done);
            break;
        case ST_BF16:
            hipLaunchKernelGGL(tail_k<bf16>, dim3(1), dim3(kNT), 0, s, D, (const bf16 *)b_in,
                               (const bf16 *)u_in, (bf16 *)u_out, has_g, done);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mg
