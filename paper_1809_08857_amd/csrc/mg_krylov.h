// BiCGStab with right preconditioning and its scalars on the device, shared
// by the solvers whose operator is not the single-grid one (composite AMR
// grids, embedded boundaries).  One host synchronisation per iteration
// reads the residual norm for the convergence test.
#pragma once

#include <functional>

#include "mg.h"
#include "mg_internal.h"

namespace mg {

struct KrylovSpace {
    hipStream_t s = nullptr;
    long n = 0;        // vector length
    long n1 = 0;       // inner products weight entries [0, n1) by w1, the rest by 1
    double w1 = 1.0;
    double *vec = nullptr;  // kKrylovVectors vectors of n
    RedWs ws{};
    double *h_pin = nullptr;
};

constexpr int kKrylovVectors = 8;  // r, r^, p, v, s, t, y, z

// Allocates and zero-fills the vectors (MG_OK or MG_ENOMEM / MG_EDEVICE).
int krylov_alloc(KrylovSpace &K, hipStream_t s, long n, long n1, double w1);
void krylov_free(KrylovSpace &K);

// y = A x; z = M^-1 v (the preconditioner may change v's entries while it
// runs but must restore them).  Both enqueue on K.s and return MG_OK or an
// error code with the message set.
using KrylovApply = std::function<int(const double *x, double *y)>;
using KrylovPrec = std::function<int(double *v, double *z)>;

// Solves A x = b from the x given, to ||b - A x|| <= rtol ||b|| (weighted
// 2-norms) in at most maxit iterations.  S receives cycles (iterations),
// rel_res0 and rel_res (the true residual of the returned x).  Returns
// MG_OK, MG_NOT_CONVERGED, or MG_EDIVERGED on a breakdown or a non-finite
// residual (message prefixed by who).  x and b are device vectors of K.n.
int bicgstab(KrylovSpace &K, const KrylovApply &A, const KrylovPrec &M, const double *b, double *x, double rtol,
             int maxit, mg_stats &S, const char *who);

// out = c1 v1 + c2 v2 (element-wise, on K.s)
hipError_t krylov_axpby(const KrylovSpace &K, double *out, double c1, const double *v1, double c2,
                        const double *v2);

}  // namespace mg
