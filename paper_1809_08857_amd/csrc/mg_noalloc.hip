// mg_residual_noalloc: the residual and norms of mg_residual for callers
// that cannot allocate device memory (code under HIP graph capture, tight
// serving loops, harnesses that forbid hipMalloc).  It needs no context:
// the operator comes with the call, and the partial sums of its reductions
// live in a file-scope device array of fixed size instead of a context's
// workspace.
#include <mutex>

#include "mg.h"
#include "mg_engine.h"

namespace mg {

// Partial sums of one reduction slot (a pair per workgroup, at most
// kMaxRedBlocks workgroups: every reduction caps its grid there and lets a
// workgroup cover several tiles) followed by the result slots.
constexpr size_t kScratchDoubles = (size_t)kMaxRedBlocks * 2 + kRedSlots;
static_assert(kScratchDoubles * sizeof(double) == MG_NOALLOC_SCRATCH_BYTES, "scratch size as documented");

static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

// Per device: the device address of `scratch` (each GPU holds its own copy).
// In host code the array's name stands for a host-side symbol, not a device
// address; only these pointers are handed to kernels.
constexpr int kMaxDevices = 64;
std::mutex g_mu;
double *g_scratch[kMaxDevices] = {};

int scratch_ptr(double **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_err(MG_EDEVICE, "mg_residual_noalloc: hipGetDevice failed: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return set_err(MG_EDEVICE, "mg_residual_noalloc: device %d is beyond the %d supported", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_err(MG_EDEVICE, "mg_residual_noalloc: hipGetSymbolAddress failed: %s", hipGetErrorString(e));
        g_scratch[dev] = static_cast<double *>(p);
    }
    *out = g_scratch[dev];
    return MG_OK;
}

#define NCK(expr)                                                                                   \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess)                                                                       \
            return set_err(MG_EDEVICE, "mg_residual_noalloc: %s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

}  // namespace
}  // namespace mg

using namespace mg;

extern "C" int mg_residual_noalloc(const mg_desc *d, const double *eps_dev, double a, const mg_bcs *bc,
                                   const double *f_dev, const double *x_dev, double *r_dev, double *rnorm,
                                   double *bnorm, void *hip_stream) {
    if (!d || !bc || !f_dev || !x_dev) return set_err(MG_EINVAL, "mg_residual_noalloc: null argument");
    if (int rc = check_grid("mg_residual_noalloc", d)) return rc;
    int mask = 0;
    if (int rc = parse_operator("mg_residual_noalloc", a, bc, &mask)) return rc;
    double *base = nullptr;
    if (int rc = scratch_ptr(&base)) return rc;
    const RedWs ws{base, base + (size_t)kMaxRedBlocks * 2};
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const size_t n = (size_t)d->nx * d->ny * d->nz;
    double h_res[2] = {0.0, 0.0};
    if (eps_dev) {  // the coefficient check of mg_set_coeffs, on the scratch
        NCK(count_bad(s, eps_dev, n, ws, 0));
        NCK(hipMemcpyAsync(h_res, ws.result, sizeof(double), hipMemcpyDeviceToHost, s));
        NCK(hipStreamSynchronize(s));
        if (h_res[0] != 0.0)
            return set_err(MG_EINVAL, "mg_residual_noalloc: %.0f coefficient entries are not in (0, 1e100]", h_res[0]);
    }
    Geo G{};
    G.nx = d->nx;
    G.ny = d->ny;
    G.nz = d->nz;
    G.bcmask = mask;
    G.h2 = d->h * d->h;
    G.a = a;
    G.ah2 = a * G.h2;
    G.ih2 = 1.0 / G.h2;
    for (int f = 0; f < 6; ++f) G.g[f] = (mask >> f & 1) ? bc->value[f] : 0.0;
    G.cw = 1.0;
    Coef C{};
    C.mode = eps_dev ? COEF_CELL : COEF_CONST;
    C.eps = eps_dev;
    if (r_dev) NCK(resid_out(s, G, C, x_dev, f_dev, r_dev));
    NCK(norm2_resid(s, ST_F64, G, C, x_dev, f_dev, ws, 0, 1));
    NCK(hipMemcpyAsync(h_res, ws.result, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    NCK(hipStreamSynchronize(s));
    if (rnorm) *rnorm = std::sqrt(h_res[0]);
    if (bnorm) *bnorm = std::sqrt(h_res[1]);
    return MG_OK;
}
