// BiCGStab (van der Vorst) with right preconditioning: the vector updates
// and inner products run in kernels that read the iteration's scalars from
// device memory, so the host enqueues a whole iteration and waits once, for
// the residual norm.
#include <cmath>

#include "mg_engine.h"
#include "mg_krylov.h"
#include "mg_stencil.cuh"

namespace mg {

namespace {

// Result slots of the reductions and the device scalars.
enum {
    S_RHO = 0,   // (r^, r)
    S_RR = 1,    // (r, r)
    S_RHV = 2,   // (r^, v); also ||b||^2 at the start
    S_TS = 3,    // (t, s)
    S_TT = 4,    // (t, t)
    S_RHO0 = 5,  // rho of the previous iteration
    S_ALPHA = 6,
    S_OMEGA = 7
};
static_assert(S_OMEGA < kRedSlots, "scalar slots");

enum { V_R = 0, V_RH, V_P, V_V, V_S, V_T, V_Y, V_Z };

// Partial pair (x1.y1, x2.y2) per workgroup into reduction slot `slot`;
// entries below n1 weigh w1.
__global__ __launch_bounds__(256) void kr_dot_k(const double *__restrict__ x1, const double *__restrict__ y1,
                                                const double *__restrict__ x2, const double *__restrict__ y2,
                                                long n1, double w1, long n, RedWs ws, int slot) {
    double s1 = 0.0, s2 = 0.0, f1 = 0.0, f2 = 0.0;
    const long stride = (long)gridDim.x * blockDim.x;
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < n1; i += stride) {
        s1 += x1[i] * y1[i];
        if (x2) s2 += x2[i] * y2[i];
    }
    for (; i < n; i += stride) {
        f1 += x1[i] * y1[i];
        if (x2) f2 += x2[i] * y2[i];
    }
    reduce2_finish<256>(w1 * s1 + f1, w1 * s2 + f2, ws, slot, blockIdx.x);
}

__device__ __forceinline__ double beta_of(const double *R) {
    const double rho0 = R[S_RHO0], om = R[S_OMEGA];
    return (rho0 != 0.0 && om != 0.0) ? (R[S_RHO] / rho0) * (R[S_ALPHA] / om) : 0.0;
}

// p = r + beta (p - omega v)
__global__ __launch_bounds__(256) void kr_p_k(double *__restrict__ p, const double *__restrict__ r,
                                              const double *__restrict__ v, const double *__restrict__ R, long n) {
    const double beta = beta_of(R), bw = beta * R[S_OMEGA];
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        p[i] = r[i] + beta * p[i] - bw * v[i];
}

// s = r - alpha v
__global__ __launch_bounds__(256) void kr_s_k(double *__restrict__ s, const double *__restrict__ r,
                                              const double *__restrict__ v, const double *__restrict__ R, long n) {
    const double al = R[S_ALPHA];
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        s[i] = r[i] - al * v[i];
}

// x += alpha y + omega z; r = s - omega t; partials of (r^, r) and (r, r)
__global__ __launch_bounds__(256) void kr_xr_k(double *__restrict__ x, const double *__restrict__ y,
                                               const double *__restrict__ z, double *__restrict__ r,
                                               const double *__restrict__ s, const double *__restrict__ t,
                                               const double *__restrict__ rh, const double *__restrict__ R,
                                               long n1, double w1, long n, RedWs ws) {
    const double al = R[S_ALPHA], om = R[S_OMEGA];
    double a1 = 0.0, a2 = 0.0, f1 = 0.0, f2 = 0.0;
    const long stride = (long)gridDim.x * blockDim.x;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        x[i] += al * y[i] + om * z[i];
        const double ri = s[i] - om * t[i];
        r[i] = ri;
        if (i < n1) {
            a1 += rh[i] * ri;
            a2 += ri * ri;
        } else {
            f1 += rh[i] * ri;
            f2 += ri * ri;
        }
    }
    reduce2_finish<256>(w1 * a1 + f1, w1 * a2 + f2, ws, S_RHO, blockIdx.x);
}

// Scalars between the reductions (one thread).  phase 0: alpha = rho /
// (r^, v); phase 1: omega = (t, s) / (t, t) and rho kept for the next
// iteration; phase 2: start values (rho0 = alpha = omega = 1).
__global__ void kr_scalar_k(double *R, int phase) {
    if (phase == 0) {
        R[S_ALPHA] = R[S_RHV] != 0.0 ? R[S_RHO] / R[S_RHV] : 0.0;
    } else if (phase == 1) {
        R[S_OMEGA] = R[S_TT] > 0.0 ? R[S_TS] / R[S_TT] : 0.0;
        R[S_RHO0] = R[S_RHO];
    } else {
        R[S_RHO0] = R[S_ALPHA] = R[S_OMEGA] = 1.0;
    }
}

__global__ void kr_axpby_k(double *out, double c1, const double *v1, double c2, const double *v2, long n) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        out[i] = c1 * v1[i] + c2 * v2[i];
}

unsigned grid1(long n) { return (unsigned)std::min<long>(std::max<long>((n + 255) / 256, 1), 16384); }
unsigned gridr(long n) { return (unsigned)std::min<long>(std::max<long>((n + 255) / 256, 1), kMaxRedBlocks); }

#define KCK(expr)                                                                                  \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return set_err(MG_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),       \
                           __FILE__, __LINE__);                                                    \
    } while (0)

double *vp(KrylovSpace &K, int k) { return K.vec + (size_t)k * K.n; }

int dot(KrylovSpace &K, const double *x1, const double *y1, const double *x2, const double *y2, int slot) {
    const unsigned nb = gridr(K.n);
    hipLaunchKernelGGL(kr_dot_k, dim3(nb), dim3(256), 0, K.s, x1, y1, x2, y2, K.n1, K.w1, K.n, K.ws, slot);
    KCK(hipGetLastError());
    KCK(reduce2_final(K.s, K.ws, slot, x2 ? slot + 1 : -1, (int)nb, -1, 0.0, nullptr, nullptr));
    return MG_OK;
}

int scalar(KrylovSpace &K, int phase) {
    hipLaunchKernelGGL(kr_scalar_k, dim3(1), dim3(1), 0, K.s, K.ws.result, phase);
    KCK(hipGetLastError());
    return MG_OK;
}

int read_slots(KrylovSpace &K) {
    KCK(hipMemcpyAsync(K.h_pin, K.ws.result, kRedSlots * sizeof(double), hipMemcpyDeviceToHost, K.s));
    KCK(hipStreamSynchronize(K.s));
    return MG_OK;
}

}  // namespace

int krylov_alloc(KrylovSpace &K, hipStream_t s, long n, long n1, double w1) {
    K.s = s;
    K.n = n;
    K.n1 = n1;
    K.w1 = w1;
    const bool ok = hipMalloc(&K.vec, sizeof(double) * kKrylovVectors * std::max<long>(n, 1)) == hipSuccess &&
                    hipMalloc(&K.ws.partials, sizeof(double) * kRedSlots * kMaxRedBlocks * 2) == hipSuccess &&
                    hipMalloc(&K.ws.result, sizeof(double) * kRedSlots) == hipSuccess &&
                    hipHostMalloc((void **)&K.h_pin, sizeof(double) * kRedSlots, hipHostMallocDefault) ==
                        hipSuccess;
    if (!ok) {
        krylov_free(K);
        return set_err(MG_ENOMEM, "Krylov workspace: device allocation failed");
    }
    if (fill_zero(s, K.vec, sizeof(double) * kKrylovVectors * n) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        krylov_free(K);
        return set_err(MG_EDEVICE, "Krylov workspace: zero fill failed");
    }
    return MG_OK;
}

void krylov_free(KrylovSpace &K) {
    for (void *p : {(void *)K.vec, (void *)K.ws.partials, (void *)K.ws.result})
        if (p) (void)hipFree(p);
    if (K.h_pin) (void)hipHostFree(K.h_pin);
    K.vec = nullptr;
    K.ws = RedWs{};
    K.h_pin = nullptr;
}

hipError_t krylov_axpby(const KrylovSpace &K, double *out, double c1, const double *v1, double c2,
                        const double *v2) {
    hipLaunchKernelGGL(kr_axpby_k, dim3(grid1(K.n)), dim3(256), 0, K.s, out, c1, v1, c2, v2, K.n);
    return hipGetLastError();
}

int bicgstab(KrylovSpace &K, const KrylovApply &A, const KrylovPrec &M, const double *b, double *x, double rtol,
             int maxit, mg_stats &S, const char *who) {
    hipStream_t s = K.s;
    const long n = K.n;
    const unsigned g1 = grid1(n), gr = gridr(n);
    double *r = vp(K, V_R), *rh = vp(K, V_RH), *p = vp(K, V_P), *v = vp(K, V_V), *sv = vp(K, V_S),
           *t = vp(K, V_T), *y = vp(K, V_Y), *z = vp(K, V_Z);
    const double *R = K.ws.result;
    int rc;
    // r = b - A x, r^ = r, p = v = 0, the start values of the scalars
    if ((rc = A(x, r))) return rc;
    KCK(krylov_axpby(K, r, 1.0, b, -1.0, r));
    KCK(hipMemcpyAsync(rh, r, n * 8, hipMemcpyDeviceToDevice, s));
    KCK(fill_zero(s, p, n * 8));
    KCK(fill_zero(s, v, n * 8));
    if ((rc = dot(K, rh, r, r, r, S_RHO)) || (rc = dot(K, b, b, nullptr, nullptr, S_RHV)) || (rc = scalar(K, 2)) ||
        (rc = read_slots(K)))
        return rc;
    const double bn = std::sqrt(K.h_pin[S_RHV]);
    S = mg_stats{};
    if (!std::isfinite(bn) || !std::isfinite(K.h_pin[S_RR]))
        return set_err(MG_EINVAL, "%s: right-hand side or initial guess is not finite", who);
    if (bn == 0.0) {
        KCK(fill_zero(s, x, n * 8));
        KCK(hipStreamSynchronize(s));
        return MG_OK;
    }
    S.rel_res0 = std::sqrt(K.h_pin[S_RR]) / bn;
    double rel = S.rel_res0;
    int it = 0, result = MG_NOT_CONVERGED;
    const char *why = nullptr;
    while (rel > rtol && it < maxit) {
        hipLaunchKernelGGL(kr_p_k, dim3(g1), dim3(256), 0, s, p, r, v, R, n);
        KCK(hipGetLastError());
        if ((rc = M(p, y)) || (rc = A(y, v)) || (rc = dot(K, rh, v, nullptr, nullptr, S_RHV)) || (rc = scalar(K, 0)))
            return rc;
        hipLaunchKernelGGL(kr_s_k, dim3(g1), dim3(256), 0, s, sv, r, v, R, n);
        KCK(hipGetLastError());
        if ((rc = M(sv, z)) || (rc = A(z, t)) || (rc = dot(K, t, sv, t, t, S_TS)) || (rc = scalar(K, 1))) return rc;
        hipLaunchKernelGGL(kr_xr_k, dim3(gr), dim3(256), 0, s, x, y, z, r, sv, t, rh, R, K.n1, K.w1, n, K.ws);
        KCK(hipGetLastError());
        KCK(reduce2_final(s, K.ws, S_RHO, S_RR, (int)gr, -1, 0.0, nullptr, nullptr));
        if ((rc = read_slots(K))) return rc;
        ++it;
        const double *H = K.h_pin;
        rel = std::sqrt(H[S_RR]) / bn;
        if (!std::isfinite(rel)) {
            why = "non-finite residual";
            break;
        }
        if (rel <= rtol) break;
        if (H[S_RHV] == 0.0 || H[S_OMEGA] == 0.0 || H[S_RHO] == 0.0) {
            why = H[S_RHV] == 0.0 ? "(r^, v) = 0" : H[S_OMEGA] == 0.0 ? "omega = 0" : "rho = 0";
            break;
        }
    }
    if (!why && rel <= rtol) {
        // the recursively updated residual drifts: confirm with the true one
        if ((rc = A(x, r))) return rc;
        KCK(krylov_axpby(K, r, 1.0, b, -1.0, r));
        if ((rc = dot(K, r, r, nullptr, nullptr, S_RR)) || (rc = read_slots(K))) return rc;
        rel = std::sqrt(K.h_pin[S_RR]) / bn;
        result = rel <= rtol * 1.01 ? MG_OK : MG_NOT_CONVERGED;
    }
    S.cycles = it;
    S.rel_res = rel;
    if (why) return set_err(MG_EDIVERGED, "%s: BiCGStab broke down (%s) after %d iterations", who, why, it);
    return result;
}

}  // namespace mg
