// Host driver of the learned initial guess (C ABI in mgl.h): the layer
// graph of the U-net, its device buffers, the forward pass, the backward
// pass (input gradients through conv(), weight gradients through wgrad()),
// Adam, prediction, training targets and parameter files.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "mgl.h"
#include "nn_internal.h"

using namespace nn;

namespace {

thread_local std::string g_err;

int set_err(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define CK(expr)                                                                                             \
    do {                                                                                                     \
        hipError_t e_ = (expr);                                                                              \
        if (e_ != hipSuccess)                                                                                \
            return set_err(MG_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__,       \
                           __LINE__);                                                                        \
    } while (0)

constexpr int kHead = -1;  // geometry tag of the 1x1 head
constexpr int kInput = -1; // input index: the scaled source
constexpr int kNone = -2;  // no second input
constexpr int kLayers = 21;
constexpr int kHeadLayer = 20;
constexpr size_t kMaxPartialFloats = size_t(32) << 20;

struct LayerDef {
    int geom;
    int cin, cout;
    int inA, inB;      // producing layers of the (concatenated) input
    int lin, lout;     // levels of the input and output grids
};

// The U-net, in the order of the parameter vector.
const LayerDef kNet[kLayers] = {
    {G_SAME3, 1, 16, kInput, kNone, 0, 0},  // e0a
    {G_SAME3, 16, 16, 0, kNone, 0, 0},      // e0b (skip 0)
    {G_DOWN2, 16, 32, 1, kNone, 0, 1},      // d0
    {G_SAME3, 32, 32, 2, kNone, 1, 1},      // e1a
    {G_SAME3, 32, 32, 3, kNone, 1, 1},      // e1b (skip 1)
    {G_DOWN2, 32, 64, 4, kNone, 1, 2},      // d1
    {G_SAME3, 64, 64, 5, kNone, 2, 2},      // e2a
    {G_SAME3, 64, 64, 6, kNone, 2, 2},      // e2b (skip 2)
    {G_DOWN2, 64, 64, 7, kNone, 2, 3},      // d2
    {G_SAME3, 64, 64, 8, kNone, 3, 3},      // b3a
    {G_SAME3, 64, 64, 9, kNone, 3, 3},      // b3b
    {G_UP2, 64, 64, 10, kNone, 3, 2},       // u2
    {G_SAME3, 128, 64, 11, 7, 2, 2},        // c2a = conv(u2 | e2b)
    {G_SAME3, 64, 64, 12, kNone, 2, 2},     // c2b
    {G_UP2, 64, 32, 13, kNone, 2, 1},       // u1
    {G_SAME3, 64, 32, 14, 4, 1, 1},         // c1a = conv(u1 | e1b)
    {G_SAME3, 32, 32, 15, kNone, 1, 1},     // c1b
    {G_UP2, 32, 16, 16, kNone, 1, 0},       // u0
    {G_SAME3, 32, 16, 17, 1, 0, 0},         // c0a = conv(u0 | e0b)
    {G_SAME3, 16, 16, 18, kNone, 0, 0},     // c0b
    {kHead, kHeadIn, 3, 19, kNone, 0, 0},   // head: c0b's 16 channels + x at 27 taps
};

int taps(const LayerDef &L) { return L.geom == kHead ? 1 : geom_taps(L.geom); }
size_t wcount(const LayerDef &L) { return (size_t)L.cout * taps(L) * L.cin; }

struct Offsets {
    size_t w[kLayers], b[kLayers], total;
    Offsets() {
        size_t o = 0;
        for (int l = 0; l < kLayers; ++l) {
            w[l] = o;
            o += wcount(kNet[l]);
            b[l] = o;
            o += kNet[l].cout;
        }
        total = o;
    }
};
const Offsets kOff;

// counter-based normal deviates: splitmix64 -> two uniforms -> Box-Muller
uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}
double normal_at(uint64_t seed, uint64_t i) {
    const double two53 = 9007199254740992.0;
    const double u1 = ((splitmix64(seed * 0x100000001B3ull + 2 * i) >> 11) + 1.0) / (two53 + 1.0);
    const double u2 = (splitmix64(seed * 0x100000001B3ull + 2 * i + 1) >> 11) / two53;
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
}

}  // namespace

struct mgl_net {
    int nx = 0, ny = 0, nz = 0;
    hipStream_t stream = nullptr;
    std::vector<void *> allocs;
    float *theta = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
    bf16_t *wf[kLayers] = {}, *wd[kLayers] = {};
    bf16_t *act[kLayers] = {}, *gact[kLayers] = {};
    bf16_t *x8 = nullptr;
    double *sigma = nullptr;       // [0]: max|s| (FP64)
    unsigned *maxbits = nullptr;   // 3 float bit patterns
    float *wpart = nullptr, *bpart = nullptr, *hpart = nullptr, *rwork = nullptr;
    float *lossacc = nullptr;
    int wslices[kLayers] = {}, bslices[kLayers] = {};
    double scale[3] = {1.0, 1.0, 1.0};
    int adam_step = 0;
    bool have_params = false;

    int dims(int lvl, int &x, int &y, int &z) const {
        x = nx >> lvl, y = ny >> lvl, z = nz >> lvl;
        return 0;
    }
    size_t cells(int lvl) const { return (size_t)(nx >> lvl) * (ny >> lvl) * (nz >> lvl); }
    void *alloc(size_t bytes) {
        void *p = nullptr;
        if (hipMalloc(&p, bytes ? bytes : 16) != hipSuccess) return nullptr;
        allocs.push_back(p);
        return p;
    }
};

namespace {

int pack_all(mgl_net *n) {
    for (int l = 0; l < kLayers; ++l) {
        const LayerDef &L = kNet[l];
        if (L.geom == kHead) continue;
        const int cinp = L.inA == kInput ? 8 : L.cin;
        CK(pack_weights(n->stream, L.geom, n->theta + kOff.w[l], L.cout, L.cin, cinp, n->wf[l],
                        l == 0 ? nullptr : n->wd[l]));
    }
    return MG_OK;
}

int reset_adam(mgl_net *n) {
    CK(fill_zero(n->stream, n->m, kOff.total * 4));
    CK(fill_zero(n->stream, n->v, kOff.total * 4));
    n->adam_step = 0;
    return MG_OK;
}

// input tensors of layer l
void inputs(const mgl_net *n, int l, const bf16_t *&a, int &ca, const bf16_t *&b, int &cb) {
    const LayerDef &L = kNet[l];
    if (L.inA == kInput) {
        a = n->x8, ca = 8;
    } else {
        a = n->act[L.inA], ca = kNet[L.inA].cout;
    }
    if (L.inB >= 0) {
        b = n->act[L.inB], cb = kNet[L.inB].cout;
    } else {
        b = nullptr, cb = 0;
    }
}

// Forward pass.  The first layer is a convolution of the padded input
// tensor x8 (channel 0 = bfloat16(s / max|s|), channels 1-7 zero), which the
// weight gradient of the first layer also reads.
int forward(mgl_net *n, const double *s) {
    hipStream_t st = n->stream;
    const size_t n0 = n->cells(0);
    CK(fill_zero(st, n->sigma, 8));
    CK(maxabs(st, s, n0, n->sigma));
    CK(prep_input(st, s, n0, n->sigma, n->x8));
    for (int l = 0; l < kLayers; ++l) {
        const LayerDef &L = kNet[l];
        if (L.geom == kHead) continue;
        ConvArgs a{};
        n->dims(L.lin, a.inx, a.iny, a.inz);
        n->dims(L.lout, a.onx, a.ony, a.onz);
        inputs(n, l, a.srcA, a.ca, a.srcB, a.cb);
        a.w = n->wf[l];
        a.bias = n->theta + kOff.b[l];
        a.relu = 1;
        a.dstA = n->act[l];
        a.da = L.cout;
        CK(conv(st, L.geom, a));
    }
    return MG_OK;
}

// head loss and gradient of one sample; sse accumulates into lossacc
int head_backward(mgl_net *n, const double *s, const float *t, bool want_grad) {
    hipStream_t st = n->stream;
    const size_t n0 = n->cells(0);
    const int nb = head_train_blocks(n->nx, n->ny, n->nz);
    constexpr int nwb = 3 * kHeadIn + 3;  // dW then db: contiguous in the parameter vector
    CK(head_train(st, n->act[19], s, n->nx, n->ny, n->nz, n->theta + kOff.w[kHeadLayer],
                  n->theta + kOff.b[kHeadLayer], n->sigma, t, n->gact[19], n->hpart));
    if (want_grad)
        CK(reduce_partials(st, n->hpart, nb, nwb, kHeadRed, nwb, nwb, n->grad + kOff.w[kHeadLayer], 1, n->rwork));
    CK(reduce_partials(st, n->hpart + nwb, nb, 1, kHeadRed, 1, 1, n->lossacc, 1, n->rwork));
    return MG_OK;
}

int backward(mgl_net *n) {
    hipStream_t st = n->stream;
    bool written[kLayers] = {};
    written[19] = true;
    for (int l = 19; l >= 0; --l) {
        const LayerDef &L = kNet[l];
        const bf16_t *xa, *xb;
        int ca, cb;
        inputs(n, l, xa, ca, xb, cb);
        // weight gradient
        WgradArgs w{};
        n->dims(L.lin, w.xnx, w.xny, w.xnz);
        n->dims(L.lout, w.gnx, w.gny, w.gnz);
        w.xA = xa, w.ca = ca, w.xB = xb, w.cb = cb;
        w.g = n->gact[l];
        w.cout = L.cout;
        w.partials = n->wpart;
        w.nslice = n->wslices[l];
        CK(wgrad(st, L.geom, w));
        const int cinp = ca + cb;
        const int T = taps(L);
        const int cnt = L.cout * T * cinp;
        CK(reduce_partials(st, n->wpart, w.nslice, cnt, cnt, cinp, L.cin, n->grad + kOff.w[l], 1, n->rwork));
        // bias gradient
        CK(bias_grad(st, n->gact[l], n->cells(L.lout), L.cout, n->bpart, n->bslices[l]));
        CK(reduce_partials(st, n->bpart, n->bslices[l], L.cout, L.cout, L.cout, L.cout, n->grad + kOff.b[l], 1, n->rwork));
        if (L.inA == kInput) continue;
        // input gradient, masked by the ReLU of each producing layer
        ConvArgs a{};
        n->dims(L.lout, a.inx, a.iny, a.inz);
        n->dims(L.lin, a.onx, a.ony, a.onz);
        a.srcA = n->gact[l];
        a.ca = L.cout;
        a.w = n->wd[l];
        a.dstA = n->gact[L.inA];
        a.da = kNet[L.inA].cout;
        a.maskA = n->act[L.inA];
        a.accA = written[L.inA];
        if (L.inB >= 0) {
            a.dstB = n->gact[L.inB];
            a.db = kNet[L.inB].cout;
            a.maskB = n->act[L.inB];
            a.accB = written[L.inB];
        }
        const int g = L.geom == G_DOWN2 ? G_UP2 : (L.geom == G_UP2 ? G_DOWN2 : G_SAME3);
        CK(conv(st, g, a));
        written[L.inA] = true;
        if (L.inB >= 0) written[L.inB] = true;
    }
    return MG_OK;
}

int check_net(const mgl_net *n, const char *fn) {
    if (!n) return set_err(MG_EINVAL, "%s: null network", fn);
    return MG_OK;
}

}  // namespace

extern "C" {

const char *mgl_last_error(void) { return g_err.c_str(); }

size_t mgl_num_params(void) { return kOff.total; }

int mgl_create(const mgl_desc *d, void *hip_stream, mgl_net **out) {
    if (!d || !out) return set_err(MG_EINVAL, "mgl_create: null argument");
    *out = nullptr;
    if (d->nx < 8 || d->ny < 8 || d->nz < 8 || d->nx % 8 || d->ny % 8 || d->nz % 8)
        return set_err(MG_EINVAL, "mgl_create: every axis must be a positive multiple of 8 (got %d x %d x %d)", d->nx,
                       d->ny, d->nz);
    if ((double)d->nx * d->ny * d->nz > 1073741824.0) return set_err(MG_EINVAL, "mgl_create: grid too large");
    mgl_net *n = new mgl_net;
    n->nx = d->nx, n->ny = d->ny, n->nz = d->nz;
    n->stream = static_cast<hipStream_t>(hip_stream);
    bool ok = true;
    auto A = [&](size_t bytes) {
        void *p = n->alloc(bytes);
        ok = ok && p;
        return p;
    };
    const size_t P = kOff.total;
    n->theta = (float *)A(P * 4);
    n->m = (float *)A(P * 4);
    n->v = (float *)A(P * 4);
    n->grad = (float *)A(P * 4);
    size_t wmax = 0, nmax = kHeadRed;
    int bmax = 0;
    for (int l = 0; l < kLayers; ++l) {
        const LayerDef &L = kNet[l];
        if (L.geom == kHead) continue;
        const int cinp = L.inA == kInput ? 8 : L.cin;
        const int T = taps(L);
        n->wf[l] = (bf16_t *)A((size_t)L.cout * T * cinp * 2);
        if (l > 0) n->wd[l] = (bf16_t *)A((size_t)L.cout * T * L.cin * 2);
        n->act[l] = (bf16_t *)A(n->cells(L.lout) * L.cout * 2);
        n->gact[l] = (bf16_t *)A(n->cells(L.lout) * L.cout * 2);
        int qx, qy, qz;
        n->dims(L.geom == G_UP2 ? L.lin : L.lout, qx, qy, qz);
        n->wslices[l] = wgrad_slices(L.geom, qx, qy, qz, cinp, L.cout, kMaxPartialFloats);
        wmax = std::max(wmax, (size_t)n->wslices[l] * L.cout * T * cinp);
        nmax = std::max(nmax, (size_t)L.cout * T * cinp);
        size_t bs = n->cells(L.lout) / 2048;
        n->bslices[l] = (int)std::min<size_t>(1024, std::max<size_t>(1, bs));
        bmax = std::max(bmax, n->bslices[l] * L.cout);
    }
    n->x8 = (bf16_t *)A(n->cells(0) * 8 * 2);
    n->sigma = (double *)A(64);
    n->maxbits = (unsigned *)A(64);
    n->lossacc = (float *)A(64);
    n->wpart = (float *)A(wmax * 4);
    n->bpart = (float *)A((size_t)bmax * 4);
    n->hpart = (float *)A((size_t)head_train_blocks(n->nx, n->ny, n->nz) * kHeadRed * 4);
    n->rwork = (float *)A(nmax * kReduceGroups * 4);
    if (!ok) {
        mgl_destroy(n);
        return set_err(MG_ENOMEM, "mgl_create: device allocation failed");
    }
    int rc;
    if (fill_zero(n->stream, n->theta, P * 4) != hipSuccess || fill_zero(n->stream, n->grad, P * 4) != hipSuccess ||
        (rc = reset_adam(n)) != MG_OK || (rc = pack_all(n)) != MG_OK ||
        hipStreamSynchronize(n->stream) != hipSuccess) {
        mgl_destroy(n);
        return set_err(MG_EDEVICE, "mgl_create: initialisation failed");
    }
    *out = n;
    return MG_OK;
}

int mgl_destroy(mgl_net *n) {
    if (!n) return MG_OK;
    (void)hipStreamSynchronize(n->stream);
    for (void *p : n->allocs) (void)hipFree(p);
    delete n;
    return MG_OK;
}

int mgl_init_params(mgl_net *n, unsigned long long seed) {
    if (int rc = check_net(n, "mgl_init_params")) return rc;
    std::vector<float> h(kOff.total, 0.f);
    uint64_t ctr = 0;
    for (int l = 0; l < kLayers; ++l) {
        const LayerDef &L = kNet[l];
        const int fan_in = L.cin * taps(L);
        const double sd = std::sqrt((L.geom == kHead ? 1.0 : 2.0) / fan_in);
        for (size_t i = 0; i < wcount(L); ++i) h[kOff.w[l] + i] = (float)(sd * normal_at(seed, ctr++));
    }
    return mgl_set_params(n, h.data(), h.size());
}

int mgl_set_params(mgl_net *n, const float *host, size_t count) {
    if (int rc = check_net(n, "mgl_set_params")) return rc;
    if (!host || count != kOff.total)
        return set_err(MG_EINVAL, "mgl_set_params: expected %zu parameters, got %zu", kOff.total, count);
    for (size_t i = 0; i < count; ++i)
        if (!std::isfinite(host[i])) return set_err(MG_EINVAL, "mgl_set_params: parameter %zu is not finite", i);
    CK(hipMemcpyAsync(n->theta, host, count * 4, hipMemcpyHostToDevice, n->stream));
    if (int rc = reset_adam(n)) return rc;
    if (int rc = pack_all(n)) return rc;
    CK(hipStreamSynchronize(n->stream));
    n->have_params = true;
    return MG_OK;
}

int mgl_get_params(mgl_net *n, float *host, size_t count) {
    if (int rc = check_net(n, "mgl_get_params")) return rc;
    if (!host || count != kOff.total) return set_err(MG_EINVAL, "mgl_get_params: expected %zu parameters", kOff.total);
    CK(hipMemcpyAsync(host, n->theta, count * 4, hipMemcpyDeviceToHost, n->stream));
    CK(hipStreamSynchronize(n->stream));
    return MG_OK;
}

int mgl_get_grads(mgl_net *n, float *host, size_t count) {
    if (int rc = check_net(n, "mgl_get_grads")) return rc;
    if (!host || count != kOff.total) return set_err(MG_EINVAL, "mgl_get_grads: expected %zu values", kOff.total);
    CK(hipMemcpyAsync(host, n->grad, count * 4, hipMemcpyDeviceToHost, n->stream));
    CK(hipStreamSynchronize(n->stream));
    return MG_OK;
}

int mgl_set_scales(mgl_net *n, const double scale[3]) {
    if (int rc = check_net(n, "mgl_set_scales")) return rc;
    if (!scale) return set_err(MG_EINVAL, "mgl_set_scales: null argument");
    for (int i = 0; i < 3; ++i)
        if (!(scale[i] > 0.0) || !std::isfinite(scale[i]))
            return set_err(MG_EINVAL, "mgl_set_scales: scale %d must be finite and > 0", i);
    for (int i = 0; i < 3; ++i) n->scale[i] = scale[i];
    return MG_OK;
}

int mgl_get_scales(const mgl_net *n, double scale[3]) {
    if (!n || !scale) return set_err(MG_EINVAL, "mgl_get_scales: null argument");
    for (int i = 0; i < 3; ++i) scale[i] = n->scale[i];
    return MG_OK;
}

int mgl_make_target(mgl_net *n, const double *s, const double *const psi[3], const double kappa2[3], float *t,
                    double maxabs_out[3]) {
    if (int rc = check_net(n, "mgl_make_target")) return rc;
    if (!s || !psi || !psi[0] || !psi[1] || !psi[2] || !kappa2 || !t)
        return set_err(MG_EINVAL, "mgl_make_target: null argument");
    for (int i = 0; i < 3; ++i)
        if (!(kappa2[i] > 0.0) || !std::isfinite(kappa2[i]))
            return set_err(MG_EINVAL, "mgl_make_target: kappa2[%d] must be finite and > 0", i);
    hipStream_t st = n->stream;
    const size_t n0 = n->cells(0);
    CK(fill_zero(st, n->sigma, 8));
    CK(fill_zero(st, n->maxbits, 16));
    CK(maxabs(st, s, n0, n->sigma));
    CK(make_target(st, psi[0], psi[1], psi[2], n0, kappa2, n->scale, n->sigma, t, n->maxbits));
    if (maxabs_out) {
        unsigned b[3];
        CK(hipMemcpyAsync(b, n->maxbits, 12, hipMemcpyDeviceToHost, st));
        CK(hipStreamSynchronize(st));
        for (int i = 0; i < 3; ++i) {
            float f;
            std::memcpy(&f, &b[i], 4);
            maxabs_out[i] = f;
        }
    }
    return MG_OK;
}

int mgl_train_step(mgl_net *n, int count, const double *const *s, const float *const *t, const mgl_adam *opt,
                   double *loss) {
    if (int rc = check_net(n, "mgl_train_step")) return rc;
    if (count < 1 || !s || !t) return set_err(MG_EINVAL, "mgl_train_step: need count >= 1 samples");
    for (int k = 0; k < count; ++k)
        if (!s[k] || !t[k]) return set_err(MG_EINVAL, "mgl_train_step: null sample %d", k);
    if (opt && (!(opt->lr >= 0.f) || !(opt->beta1 >= 0.f && opt->beta1 < 1.f) ||
                !(opt->beta2 >= 0.f && opt->beta2 < 1.f) || !(opt->eps > 0.f)))
        return set_err(MG_EINVAL, "mgl_train_step: invalid Adam parameters");
    hipStream_t st = n->stream;
    CK(fill_zero(st, n->grad, kOff.total * 4));
    CK(fill_zero(st, n->lossacc, 4));
    for (int k = 0; k < count; ++k) {
        if (int rc = forward(n, s[k])) return rc;
        if (int rc = head_backward(n, s[k], t[k], true)) return rc;
        if (int rc = backward(n)) return rc;
    }
    if (opt && opt->lr > 0.f) {
        n->adam_step++;
        CK(adam(st, n->theta, n->m, n->v, n->grad, kOff.total, 1.f / count, opt->lr, opt->beta1, opt->beta2,
                opt->eps, n->adam_step));
        if (int rc = pack_all(n)) return rc;
    }
    if (loss) {
        float l;
        CK(hipMemcpyAsync(&l, n->lossacc, 4, hipMemcpyDeviceToHost, st));
        CK(hipStreamSynchronize(st));
        *loss = (double)l / (3.0 * (double)n->cells(0) * count);
    }
    return MG_OK;
}

int mgl_eval_loss(mgl_net *n, const double *s, const float *t, double *loss) {
    if (int rc = check_net(n, "mgl_eval_loss")) return rc;
    if (!s || !t || !loss) return set_err(MG_EINVAL, "mgl_eval_loss: null argument");
    hipStream_t st = n->stream;
    CK(fill_zero(st, n->lossacc, 4));
    if (int rc = forward(n, s)) return rc;
    if (int rc = head_backward(n, s, t, false)) return rc;
    float l;
    CK(hipMemcpyAsync(&l, n->lossacc, 4, hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    *loss = (double)l / (3.0 * (double)n->cells(0));
    return MG_OK;
}

int mgl_predict(mgl_net *n, const double *s, const double kappa2[3], double *const guess[3]) {
    if (int rc = check_net(n, "mgl_predict")) return rc;
    if (!s || !kappa2 || !guess || !guess[0] || !guess[1] || !guess[2])
        return set_err(MG_EINVAL, "mgl_predict: null argument");
    double coef[3];
    for (int i = 0; i < 3; ++i) {
        if (!(kappa2[i] > 0.0) || !std::isfinite(kappa2[i]))
            return set_err(MG_EINVAL, "mgl_predict: kappa2[%d] must be finite and > 0", i);
        coef[i] = n->scale[i] / kappa2[i];
    }
    if (int rc = forward(n, s)) return rc;
    CK(head_predict(n->stream, n->act[19], s, n->nx, n->ny, n->nz, n->theta + kOff.w[kHeadLayer],
                    n->theta + kOff.b[kHeadLayer], n->sigma, coef, guess[0], guess[1], guess[2]));
    return MG_OK;
}

int mgl_save(mgl_net *n, const char *path) {
    if (int rc = check_net(n, "mgl_save")) return rc;
    if (!path) return set_err(MG_EINVAL, "mgl_save: null path");
    std::vector<float> h(kOff.total);
    if (int rc = mgl_get_params(n, h.data(), h.size())) return rc;
    FILE *f = std::fopen(path, "wb");
    if (!f) return set_err(MG_EINVAL, "mgl_save: cannot open %s", path);
    const char magic[4] = {'M', 'G', 'L', 'W'};
    const uint32_t version = 1;
    const uint64_t cnt = kOff.total;
    bool ok = std::fwrite(magic, 1, 4, f) == 4 && std::fwrite(&version, 4, 1, f) == 1 &&
              std::fwrite(&cnt, 8, 1, f) == 1 && std::fwrite(n->scale, 8, 3, f) == 3 &&
              std::fwrite(h.data(), 4, h.size(), f) == h.size();
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) return set_err(MG_EINVAL, "mgl_save: write to %s failed", path);
    return MG_OK;
}

int mgl_load(mgl_net *n, const char *path) {
    if (int rc = check_net(n, "mgl_load")) return rc;
    if (!path) return set_err(MG_EINVAL, "mgl_load: null path");
    FILE *f = std::fopen(path, "rb");
    if (!f) return set_err(MG_EINVAL, "mgl_load: cannot open %s", path);
    char magic[4];
    uint32_t version = 0;
    uint64_t cnt = 0;
    double sc[3];
    std::vector<float> h(kOff.total);
    bool ok = std::fread(magic, 1, 4, f) == 4 && std::memcmp(magic, "MGLW", 4) == 0 &&
              std::fread(&version, 4, 1, f) == 1 && version == 1 && std::fread(&cnt, 8, 1, f) == 1 &&
              cnt == kOff.total && std::fread(sc, 8, 3, f) == 3 && std::fread(h.data(), 4, h.size(), f) == h.size();
    std::fclose(f);
    if (!ok) return set_err(MG_EINVAL, "mgl_load: %s is not a parameter file of this network", path);
    if (int rc = mgl_set_scales(n, sc)) return rc;
    return mgl_set_params(n, h.data(), h.size());
}

int mgl_tensor_shape(const mgl_net *n, int layer, int dims[4]) {
    if (!n || !dims) return set_err(MG_EINVAL, "mgl_tensor_shape: null argument");
    if (layer < -1 || layer >= kHeadLayer) return set_err(MG_EINVAL, "mgl_tensor_shape: no layer %d", layer);
    const int lvl = layer < 0 ? 0 : kNet[layer].lout;
    dims[0] = n->nz >> lvl, dims[1] = n->ny >> lvl, dims[2] = n->nx >> lvl;
    dims[3] = layer < 0 ? 8 : kNet[layer].cout;
    return MG_OK;
}

int mgl_read_tensor(mgl_net *n, int which, int layer, float *host, size_t count) {
    int d[4];
    if (int rc = mgl_tensor_shape(n, layer, d)) return rc;
    if (which != 0 && which != 1) return set_err(MG_EINVAL, "mgl_read_tensor: which must be 0 or 1");
    if (layer < 0 && which != 0) return set_err(MG_EINVAL, "mgl_read_tensor: the input has no gradient");
    const size_t cnt = (size_t)d[0] * d[1] * d[2] * d[3];
    if (!host || count != cnt) return set_err(MG_EINVAL, "mgl_read_tensor: expected %zu values", cnt);
    const bf16_t *src = layer < 0 ? n->x8 : (which ? n->gact[layer] : n->act[layer]);
    float *tmp = nullptr;
    CK(hipMalloc(&tmp, cnt * 4));
    hipError_t e = bf16_to_f32(n->stream, src, tmp, cnt);
    if (e == hipSuccess) e = hipMemcpyAsync(host, tmp, cnt * 4, hipMemcpyDeviceToHost, n->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
    (void)hipFree(tmp);
    CK(e);
    return MG_OK;
}

}  // extern "C"
