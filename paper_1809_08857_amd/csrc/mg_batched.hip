// Batched solves: many independent problems (different sizes and
// coefficients) advance together.
//
// Every phase of a V-cycle (one smoothing sweep of depth d, a residual
// restriction, a prolongation, the bottom solve, the FP64 refinement update)
// is ONE kernel launch over a work table of (problem, tile) entries covering
// all problems that have that phase; each workgroup reads its problem's
// descriptor and runs the same device code as the single-problem kernels.
// Each problem has its own convergence flag, set by its own deterministic
// residual reduction, and every workgroup of a converged problem returns at
// once.  One refinement step (inner low-precision V-cycle + FP64 update) is
// captured into a hipGraph (one per parity of the x / spare buffers) and
// replayed until every flag is set.  The smoother tile shape of each phase
// is picked by timing the candidates when the plan is built.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "mg_engine.h"
#include "mg_ir.cuh"
#include "mg_stencil.cuh"

namespace mg {

struct WorkRef {
    int item;  // descriptor index
    int blk;   // block index within that problem's launch
};

template <class T> struct BSmooth {
    SmoothArgs<T> a;
    int mode, zin;
};

template <class T> struct BRr {
    RrArgs<T> a;
    int mode;
};

template <class T> struct BProlong {
    T *u;
    const T *e;
    Geo G, Gc;
    int gx, gy;  // brick blocks along x (coarse columns / 32) and y (rows / 8)
    const int *done;
};

// FP64 refinement pass of one problem: xn = x + e (or 0 / x), r = b - A xn
// cast to the inner storage type, ||r||^2 (and ||b||^2) reduced per problem.
template <class TL> struct BIr {
    const double *x;
    const TL *e;
    double *xout;
    const double *f;
    const double *eps;
    Geo G;
    int mode;
    TL *rl;
    RedWs ws;
    int slot, bslot, ref_slot;
    double rtol2;
    int *done;
    int gx, gy, kz, nblk;  // column-kernel tiles in x and y, planes per z chunk, tiles
    int nwg;               // workgroups (each covers the tiles q, q + nwg, ...)
    int has_e, zero_x;
    double sc0;            // > 0: cast scale of this pass, else ws.result[2] (residual scaling)
    double cs;             // power of two multiplying the inner operator's coefficients
    double ncell;
};

constexpr int kBX = 32, kBY = 8;  // brick block of the batched element-wise kernels

// ------------------------------------------------------------ kernels

template <class T, int TX, int TY, int PD>
__global__ __launch_bounds__((TX + 4) / 2 * (TY + 4)) void b_smooth_k(const BSmooth<T> *__restrict__ items,
                                                                      const WorkRef *__restrict__ work,
                                                                      int nwork) {
    const WorkRef r = work[xcd_remap(blockIdx.x, nwork)];
    const BSmooth<T> &it = items[r.item];  // read in place: a local copy would live in scratch
    if (it.a.done && *it.a.done) return;
    __shared__ typename Num<T>::C smem[smooth_lds<COEF_CELL, TX, TY>()];
    const bool ev = (it.a.G.nx & 1) == 0;  // rows of even length: wide pair accesses
    switch (it.mode * 2 + it.zin) {
        case 0:
            if (ev) rbgs_col_body<T, COEF_CONST, TX, TY, false, PD, true>(it.a, r.blk, smem);
            else rbgs_col_body<T, COEF_CONST, TX, TY, false, PD, false>(it.a, r.blk, smem);
            break;
        case 1:
            if (ev) rbgs_col_body<T, COEF_CONST, TX, TY, true, PD, true>(it.a, r.blk, smem);
            else rbgs_col_body<T, COEF_CONST, TX, TY, true, PD, false>(it.a, r.blk, smem);
            break;
        case 2:
            if (ev) rbgs_col_body<T, COEF_CELL, TX, TY, false, PD, true>(it.a, r.blk, smem);
            else rbgs_col_body<T, COEF_CELL, TX, TY, false, PD, false>(it.a, r.blk, smem);
            break;
        case 3:
            if (ev) rbgs_col_body<T, COEF_CELL, TX, TY, true, PD, true>(it.a, r.blk, smem);
            else rbgs_col_body<T, COEF_CELL, TX, TY, true, PD, false>(it.a, r.blk, smem);
            break;
        // stored faces: the general pair body, whose register footprint is
        // close to the other two; the streaming face body of the single
        // engine would set this kernel's register count for every case
        case 4: rbgs_pair_body<T, COEF_FACE, TX, TY, false, PD>(it.a, r.blk, smem); break;
        default: rbgs_pair_body<T, COEF_FACE, TX, TY, true, PD>(it.a, r.blk, smem); break;
    }
}

template <class T, int TX, int TY, int PD>
__global__ __launch_bounds__((rr_threads<TX, TY>())) void b_rr_k(const BRr<T> *__restrict__ items,
                                                                 const WorkRef *__restrict__ work,
                                                                 int nwork) {
    const WorkRef r = work[xcd_remap(blockIdx.x, nwork)];
    const BRr<T> &it = items[r.item];  // read in place: a local copy would live in scratch
    if (it.a.done_in && *it.a.done_in) return;
    __shared__ typename Num<T>::C smem[rr_lds<COEF_CELL, TX, TY>()];
    switch (it.mode) {
        case COEF_CONST: rr_col_body<T, COEF_CONST, TX, TY, PD>(it.a, r.blk, smem); break;
        case COEF_CELL: rr_col_body<T, COEF_CELL, TX, TY, PD>(it.a, r.blk, smem); break;
        default: rr_col_body<T, COEF_FACE, TX, TY, PD>(it.a, r.blk, smem); break;
    }
}

template <class T>
__global__ __launch_bounds__(kBX *kBY) void b_prolong_k(const BProlong<T> *__restrict__ items,
                                                        const WorkRef *__restrict__ work) {
    const WorkRef r = work[blockIdx.x];
    const BProlong<T> &it = items[r.item];
    if (it.done && *it.done) return;
    const int bx = r.blk % it.gx, rest = r.blk / it.gx;
    const int by = rest % it.gy, bz = rest / it.gy;
    prolong_body<T, T>(it.u, it.e, it.G, it.Gc, bx * kBX + threadIdx.x, by * kBY + threadIdx.y, bz);
}

// FP64 refinement pass of every problem: the single engine's column kernel
// body, one workgroup per (problem, tile and z chunk).
constexpr int kIrTX = 64, kIrTY = 4;

// Final sums of the refinement pass: workgroup i finishes problem i.
template <class TL>
__global__ __launch_bounds__(kFinalThreads) void b_ir_final_k(const BIr<TL> *__restrict__ items, int check_done) {
    const BIr<TL> &it = items[blockIdx.x];
    if (check_done && it.done && *it.done) return;
    ir_final_body(it.ws, it.slot, it.bslot, it.nwg, it.ref_slot, it.rtol2, it.done, it.ws.result + 2, it.sc0,
                  it.ncell);
}

template <class TL>
__global__ __launch_bounds__(kIrTX *kIrTY) void b_ir_k(const BIr<TL> *__restrict__ items,
                                                       const WorkRef *__restrict__ work, int check_done) {
    const WorkRef r = work[blockIdx.x];
    const BIr<TL> it = items[r.item];
    if (check_done && it.done && *it.done) return;
#define MG_B_IR(MODE, HE)                                                                                      \
    ir_tiles<TL, MODE, HE, kIrTX, kIrTY, false>(it.x, it.e, it.xout, it.f, it.eps, it.G, it.rl, it.ws, it.slot,  \
                                                it.bslot, it.kz, it.gx, it.gy, r.blk, it.nblk, it.nwg, r.blk,   \
                                                it.zero_x != 0, it.ws.result + 2, it.sc0, it.cs)
    if (it.mode == COEF_CELL) {
        if (it.has_e) MG_B_IR(COEF_CELL, true);
        else MG_B_IR(COEF_CELL, false);
    } else {
        if (it.has_e) MG_B_IR(COEF_CONST, true);
        else MG_B_IR(COEF_CONST, false);
    }
#undef MG_B_IR
}

// ------------------------------------------------------------ plan

namespace {

struct Launch {
    enum Kind { SMOOTH, RR, PROLONG, TAIL } kind;
    int tile;      // smoother tile variant: 0 = 64x8, 1 = 32x8, 2 = 16x8
    size_t items;  // byte offset of the descriptor array in the plan buffer
    size_t work;   // byte offset of the work table
    int nwork;     // blocks of the launch (TAIL: problems)
    size_t descs;  // TAIL: offset of the TailDesc array
};

constexpr int kBatchTiles[3][2] = {{64, 8}, {32, 8}, {16, 8}};

template <class T>
hipError_t launch_phase(hipStream_t s, const Launch &L, char *base, int st) {
    if (L.nwork <= 0) return hipSuccess;
    const WorkRef *work = reinterpret_cast<const WorkRef *>(base + L.work);
    switch (L.kind) {
        case Launch::SMOOTH: {
            const BSmooth<T> *it = reinterpret_cast<const BSmooth<T> *>(base + L.items);
            if (L.tile == 0)
                hipLaunchKernelGGL((b_smooth_k<T, 64, 8, kSmoothPD>), dim3(L.nwork), dim3(34 * 12), 0, s, it, work, L.nwork);
            else if (L.tile == 1)
                hipLaunchKernelGGL((b_smooth_k<T, 32, 8, kSmoothPD>), dim3(L.nwork), dim3(18 * 12), 0, s, it, work, L.nwork);
            else
                hipLaunchKernelGGL((b_smooth_k<T, 16, 8, kSmoothPD>), dim3(L.nwork), dim3(10 * 12), 0, s, it, work, L.nwork);
            break;
        }
        case Launch::RR: {
            const BRr<T> *it = reinterpret_cast<const BRr<T> *>(base + L.items);
            if (L.tile == 0)
                hipLaunchKernelGGL((b_rr_k<T, 64, 8, kSmoothPD>), dim3(L.nwork), dim3(rr_threads<64, 8>()), 0, s, it, work, L.nwork);
            else if (L.tile == 1)
                hipLaunchKernelGGL((b_rr_k<T, 32, 8, kSmoothPD>), dim3(L.nwork), dim3(rr_threads<32, 8>()), 0, s, it, work, L.nwork);
            else
                hipLaunchKernelGGL((b_rr_k<T, 16, 8, kSmoothPD>), dim3(L.nwork), dim3(rr_threads<16, 8>()), 0, s, it, work, L.nwork);
            break;
        }
        case Launch::PROLONG:
            hipLaunchKernelGGL(b_prolong_k<T>, dim3(L.nwork), dim3(kBX, kBY), 0, s,
                               reinterpret_cast<const BProlong<T> *>(base + L.items), work);
            break;
        case Launch::TAIL:
            return tail_solve_batched(s, st, reinterpret_cast<const TailDesc *>(base + L.descs),
                                      reinterpret_cast<const TailIo *>(base + L.items), L.nwork);
    }
    return hipGetLastError();
}

hipError_t launch_phase_st(hipStream_t s, const Launch &L, char *base, int st) {
    switch (st) {
        case ST_F64: return launch_phase<double>(s, L, base, st);
        case ST_F32: return launch_phase<float>(s, L, base, st);
        case ST_BF16: return launch_phase<bf16>(s, L, base, st);
    }
    return hipErrorInvalidValue;
}

template <class TL>
hipError_t launch_ir(hipStream_t s, char *base, size_t items, size_t work, int nwork, int count, bool check_done) {
    if (nwork <= 0) return hipSuccess;
    hipLaunchKernelGGL(b_ir_k<TL>, dim3(nwork), dim3(kIrTX * kIrTY), 0, s,
                       reinterpret_cast<const BIr<TL> *>(base + items), reinterpret_cast<const WorkRef *>(base + work),
                       check_done ? 1 : 0);
    if (hipPeekAtLastError() != hipSuccess) return hipGetLastError();
    hipLaunchKernelGGL(b_ir_final_k<TL>, dim3(count), dim3(kFinalThreads), 0, s,
                       reinterpret_cast<const BIr<TL> *>(base + items), check_done ? 1 : 0);
    return hipGetLastError();
}

// Host image of the plan's device buffer: appended blobs, 256-byte aligned.
struct Blob {
    std::vector<char> bytes;
    template <class X> size_t add(const std::vector<X> &v) {
        size_t off = (bytes.size() + 255) / 256 * 256;
        bytes.resize(off + v.size() * sizeof(X));
        if (!v.empty()) std::memcpy(bytes.data() + off, v.data(), v.size() * sizeof(X));
        return off;
    }
};

}  // namespace

struct BatchPlan {
    std::vector<const Ctx *> ctxs;
    std::vector<unsigned> versions;
    std::vector<const double *> fs;
    std::vector<double *> xs;
    int st = -1;
    int count = 0;
    hipStream_t stream = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    char *dbuf = nullptr;        // descriptors and work tables
    int *flags = nullptr;        // per-problem convergence flags (device)
    int *h_flags = nullptr;      // pinned copies
    double *h_res = nullptr;
    int *h_one = nullptr;        // pinned constant 1 (stops a diverged problem)
    double *partials = nullptr;  // per-problem reduction workspace
    double *results = nullptr;   // per problem: [0] ||r||^2, [1] ||b||^2
    std::vector<Launch> cycle;   // inner V-cycle phases
    // [0],[1]: parities; [2],[3]: initial pass (zero x / guess) with unit
    // residual scale; [4],[5]: the same passes with the scale of the slot
    size_t ir_items[6] = {0, 0, 0, 0, 0, 0}, ir_work = 0;
    int ir_nwork = 0;
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    std::vector<double *> xalt;
    std::vector<unsigned long> uids;
};

static void plan_free(BatchPlan *p) {
    if (!p) return;
    for (int q = 0; q < 2; ++q)
        if (p->graph[q]) (void)hipGraphExecDestroy(p->graph[q]);
    if (p->dbuf) (void)hipFree(p->dbuf);
    if (p->flags) (void)hipFree(p->flags);
    if (p->partials) (void)hipFree(p->partials);
    if (p->results) (void)hipFree(p->results);
    if (p->h_flags) (void)hipHostFree(p->h_flags);
    if (p->h_res) (void)hipHostFree(p->h_res);
    if (p->h_one) (void)hipHostFree(p->h_one);
    if (p->ev_in) (void)hipEventDestroy(p->ev_in);
    if (p->ev_out) (void)hipEventDestroy(p->ev_out);
    if (p->stream) (void)hipStreamDestroy(p->stream);
    delete p;
}

void batch_release(Ctx *c) {
    plan_free(c->plan);
    c->plan = nullptr;
}

#define BCK(expr)                                                                                  \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return set_err(MG_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),       \
                           __FILE__, __LINE__);                                                    \
    } while (0)

template <class T>
static SmoothArgs<T> smooth_args(const LvView &W, int tx, int ty, const int *done, int *nblk_out) {
    SmoothArgs<T> a{};
    a.uin = static_cast<const T *>(W.u);
    a.uout = static_cast<T *>(W.t);
    a.b = static_cast<const T *>(W.b);
    a.eps = static_cast<const coef_t<T> *>(W.C.eps);
    a.fbx = static_cast<const coef_t<T> *>(W.C.bx);
    a.fby = static_cast<const coef_t<T> *>(W.C.by);
    a.fbz = static_cast<const coef_t<T> *>(W.C.bz);
    a.G = W.G;
    a.tiles_x = (W.G.nx + tx - 1) / tx;
    a.tiles_y = (W.G.ny + ty - 1) / ty;
    const int cols = a.tiles_x * a.tiles_y;
    int chunks = std::max(1, std::min((256 + cols - 1) / cols, std::max(1, W.G.nz / 8)));
    a.cz = (W.G.nz + chunks - 1) / chunks;
    a.nblk = cols * ((W.G.nz + a.cz - 1) / a.cz);
    a.done = done;
    *nblk_out = a.nblk;
    return a;
}

template <class T>
static RrArgs<T> rr_args(const LvView &W, const LvView &Wc, int tx, int ty, const int *done, int *nblk_out) {
    RrArgs<T> a{};
    a.u = static_cast<const T *>(W.u);
    a.b = static_cast<const T *>(W.b);
    a.eps = static_cast<const coef_t<T> *>(W.C.eps);
    a.fbx = static_cast<const coef_t<T> *>(W.C.bx);
    a.fby = static_cast<const coef_t<T> *>(W.C.by);
    a.fbz = static_cast<const coef_t<T> *>(W.C.bz);
    a.G = W.G;
    a.bc = static_cast<T *>(Wc.bw);
    a.tiles_x = (W.G.nx + tx - 1) / tx;
    a.tiles_y = (W.G.ny + ty - 1) / ty;
    const int cols = a.tiles_x * a.tiles_y;
    int chunks = std::max(1, std::min((256 + cols - 1) / cols, std::max(1, W.G.nz / 8)));
    int cz = (W.G.nz + chunks - 1) / chunks;
    cz += cz & 1;
    a.cz = cz;
    a.nblk = cols * ((W.G.nz + cz - 1) / cz);
    a.slot = -1;
    a.ref_slot = -1;
    a.done_in = done;
    *nblk_out = a.nblk;
    return a;
}

// Build the plan: the phase list of one inner V-cycle over all problems,
// the FP64 refinement passes, and the two captured step graphs.
template <class T, class TL>
static int build_plan(BatchPlan *P, int count, mg_ctx *const *c, const double *const *f, double *const *x) {
    const int nu1 = c[0]->d.nu1, nu2 = c[0]->d.nu2;
    std::vector<std::vector<LvView>> V(count);
    int depth = 0;
    for (int i = 0; i < count; ++i) {
        lowp_view(c[i], V[i]);
        depth = std::max(depth, c[i]->tail);
    }
    Blob blob;
    // --- down: smoothing sweeps and restrictions per depth
    auto tile_for_depth = [&](int d) {
        int mn = 1 << 30;
        for (int i = 0; i < count; ++i)
            if (d < c[i]->tail) mn = std::min(mn, V[i][d].G.nx);
        return mn >= 64 ? 0 : (mn >= 32 ? 1 : 2);
    };
    // a smoothing phase gets one work table per candidate tile; the fastest
    // is kept after timing (cands[] below)
    std::vector<std::array<Launch, 3>> cands;
    std::vector<int> cand_phase;
    auto add_smooth = [&](int d, bool zin) {
        std::array<Launch, 3> cl;
        for (int tile = 0; tile < 3; ++tile) {
            const int tx = kBatchTiles[tile][0], ty = kBatchTiles[tile][1];
            std::vector<BSmooth<T>> items;
            std::vector<WorkRef> work;
            for (int i = 0; i < count; ++i) {
                if (d >= c[i]->tail) continue;
                const LvView &W = V[i][d];
                int nb;
                BSmooth<T> it{};
                it.a = smooth_args<T>(W, tx, ty, P->flags + i, &nb);
                it.mode = W.C.mode;
                it.zin = zin ? 1 : 0;
                for (int q = 0; q < nb; ++q) work.push_back(WorkRef{(int)items.size(), q});
                items.push_back(it);
            }
            cl[tile] = Launch{Launch::SMOOTH, tile, blob.add(items), blob.add(work), (int)work.size(), 0};
        }
        for (int i = 0; i < count; ++i)
            if (d < c[i]->tail) std::swap(V[i][d].u, V[i][d].t);
        cand_phase.push_back((int)P->cycle.size());
        cands.push_back(cl);
        P->cycle.push_back(cl[tile_for_depth(d)]);
    };
    for (int d = 0; d < depth; ++d) {
        for (int q = 0; q < nu1; ++q) add_smooth(d, q == 0);
        const int tile = tile_for_depth(d);
        const int tx = kBatchTiles[tile][0], ty = kBatchTiles[tile][1];
        std::vector<BRr<T>> items;
        std::vector<WorkRef> work;
        for (int i = 0; i < count; ++i) {
            if (d >= c[i]->tail) continue;
            int nb;
            BRr<T> it{};
            it.a = rr_args<T>(V[i][d], V[i][d + 1], tx, ty, P->flags + i, &nb);
            it.mode = V[i][d].C.mode;
            for (int q = 0; q < nb; ++q) work.push_back(WorkRef{(int)items.size(), q});
            items.push_back(it);
        }
        P->cycle.push_back(Launch{Launch::RR, tile, blob.add(items), blob.add(work), (int)work.size(), 0});
    }
    // --- bottom solves, one workgroup per problem
    {
        std::vector<TailDesc> descs(count);
        std::vector<TailIo> io(count);
        for (int i = 0; i < count; ++i) {
            descs[i] = c[i]->tails[0];
            LvView &W = V[i][c[i]->tail];
            io[i] = TailIo{W.b, W.u, P->flags + i};
        }
        Launch L{Launch::TAIL, 0, blob.add(io), 0, count, blob.add(descs)};
        P->cycle.push_back(L);
    }
    // --- up: prolongation and smoothing sweeps per depth
    for (int d = depth - 1; d >= 0; --d) {
        std::vector<BProlong<T>> items;
        std::vector<WorkRef> work;
        for (int i = 0; i < count; ++i) {
            if (d >= c[i]->tail) continue;
            LvView &W = V[i][d], &Wc = V[i][d + 1];
            BProlong<T> it{};
            it.u = static_cast<T *>(W.u);
            it.e = static_cast<const T *>(Wc.u);
            it.G = W.G;
            it.Gc = Wc.G;
            it.gx = (Wc.G.nx + kBX - 1) / kBX;
            it.gy = (W.G.ny + kBY - 1) / kBY;
            it.done = P->flags + i;
            const int nb = it.gx * it.gy * W.G.nz;
            for (int q = 0; q < nb; ++q) work.push_back(WorkRef{(int)items.size(), q});
            items.push_back(it);
        }
        P->cycle.push_back(Launch{Launch::PROLONG, 0, blob.add(items), blob.add(work), (int)work.size(), 0});
        for (int q = 0; q < nu2; ++q) add_smooth(d, false);
    }
    // --- FP64 refinement passes: [0] x -> xalt, [1] xalt -> x, [2] initial
    {
        std::vector<BIr<TL>> it[6];
        std::vector<WorkRef> work;
        // Workgroups of the whole pass: about 32 per CU, shared out by cell
        // count, so that each marches a long column: a workgroup of a few
        // planes spends most of its time loading the planes around its
        // chunk and in the closing reduction.
        int cus = 256;
        {
            int dev = 0, v = 0;
            if (hipGetDevice(&dev) == hipSuccess &&
                hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
                cus = v;
        }
        double cells_all = 0.0;
        for (int i = 0; i < count; ++i) cells_all += (double)c[i]->L[0].n;
        const double budget = 32.0 * cus;
        for (int i = 0; i < count; ++i) {
            Ctx *ci = c[i];
            const Geo G0 = level_geo(ci, 0, true);
            BIr<TL> b{};
            b.f = f[i];
            b.eps = ci->has_eps ? ci->eps : nullptr;
            b.G = G0;
            b.mode = ci->has_eps ? COEF_CELL : COEF_CONST;
            b.rl = static_cast<TL *>(V[i][0].bw);
            b.ws = RedWs{P->partials + (size_t)i * kMaxRedBlocks * 2, P->results + 4 * i};
            b.slot = 0;
            b.ref_slot = 1;
            b.rtol2 = ci->d.rtol * ci->d.rtol;
            b.done = P->flags + i;
            // tiles of the column kernel and z chunks; at most kMaxRedBlocks
            // workgroups per problem, each covering several tiles of planes
            // wider than that
            b.gx = (G0.nx + kIrTX - 1) / kIrTX;
            b.gy = (G0.ny + kIrTY - 1) / kIrTY;
            const int cols = b.gx * b.gy;
            const int room = std::max(1, kMaxRedBlocks / cols);
            const double want = budget * (double)ci->L[0].n / cells_all;
            const int gz = std::max(1, std::min({G0.nz, room, (int)std::ceil(want / cols)}));
            b.kz = (G0.nz + gz - 1) / gz;
            b.nblk = b.gx * b.gy * ((G0.nz + b.kz - 1) / b.kz);
            b.nwg = std::min(b.nblk, kMaxRedBlocks);
            b.sc0 = 0.0;
            b.cs = ci->cscale;
            b.ncell = (double)ci->L[0].n;
            b.has_e = 1;
            b.zero_x = 0;
            b.bslot = -1;
            // the inner V-cycle leaves its result in the pointer the level-0 view ends on
            b.e = static_cast<const TL *>(V[i][0].u);
            BIr<TL> b0 = b, b1 = b, b2 = b;
            b0.x = x[i];
            b0.xout = P->xalt[i];
            b1.x = P->xalt[i];
            b1.xout = x[i];
            b2.x = x[i];
            b2.xout = x[i];
            b2.e = nullptr;
            b2.has_e = 0;
            b2.bslot = 1;
            b2.sc0 = 1.0;
            BIr<TL> b3 = b2;
            b2.zero_x = 1;
            BIr<TL> b4 = b2, b5 = b3;
            b4.sc0 = 0.0;
            b5.sc0 = 0.0;
            for (int q = 0; q < b.nwg; ++q) work.push_back(WorkRef{(int)it[0].size(), q});
            it[0].push_back(b0);
            it[1].push_back(b1);
            it[2].push_back(b2);
            it[3].push_back(b3);
            it[4].push_back(b4);
            it[5].push_back(b5);
        }
        for (int q = 0; q < 6; ++q) P->ir_items[q] = blob.add(it[q]);
        P->ir_work = blob.add(work);
        P->ir_nwork = (int)work.size();
    }
    BCK(hipMalloc(&P->dbuf, blob.bytes.size()));
    BCK(hipMemcpyAsync(P->dbuf, blob.bytes.data(), blob.bytes.size(), hipMemcpyHostToDevice, P->stream));
    BCK(hipStreamSynchronize(P->stream));
    // --- pick the smoother tile of each sweep phase by timing the candidates
    // (the sweeps only touch the inner cycle's scratch arrays)
    {
        hipEvent_t e0, e1;
        BCK(hipEventCreate(&e0));
        BCK(hipEventCreate(&e1));
        BCK(hipMemsetAsync(P->flags, 0, sizeof(int) * count, P->stream));
        for (size_t q = 0; q < cands.size(); ++q) {
            float best_ms = 1e30f;
            int best = P->cycle[cand_phase[q]].tile;
            for (int cand = 0; cand < 3; ++cand) {
                const Launch &L = cands[q][cand];
                BCK(launch_phase_st(P->stream, L, P->dbuf, P->st));
                BCK(hipEventRecord(e0, P->stream));
                for (int rep = 0; rep < 2; ++rep) BCK(launch_phase_st(P->stream, L, P->dbuf, P->st));
                BCK(hipEventRecord(e1, P->stream));
                BCK(hipEventSynchronize(e1));
                float ms;
                BCK(hipEventElapsedTime(&ms, e0, e1));
                if (ms < best_ms) {
                    best_ms = ms;
                    best = cand;
                }
            }
            P->cycle[cand_phase[q]] = cands[q][best];
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    // --- capture one refinement step per parity
    for (int par = 0; par < 2; ++par) {
        hipGraph_t g = nullptr;
        BCK(hipStreamBeginCapture(P->stream, hipStreamCaptureModeThreadLocal));
        hipError_t err = hipSuccess;
        for (const Launch &L : P->cycle)
            if (err == hipSuccess) err = launch_phase_st(P->stream, L, P->dbuf, P->st);
        if (err == hipSuccess) err = launch_ir<TL>(P->stream, P->dbuf, P->ir_items[par], P->ir_work, P->ir_nwork, P->count, true);
        hipError_t e2 = hipStreamEndCapture(P->stream, &g);
        if (err != hipSuccess || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return set_err(MG_EDEVICE, "mg_solve_batched: graph capture failed (%s)",
                           hipGetErrorString(err != hipSuccess ? err : e2));
        }
        hipError_t e3 = hipGraphInstantiate(&P->graph[par], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e3 != hipSuccess) return set_err(MG_EDEVICE, "mg_solve_batched: graph instantiation failed");
    }
    return MG_OK;
}

static bool plan_matches(const BatchPlan *P, int count, mg_ctx *const *c, const double *const *f,
                         double *const *x) {
    if (!P || P->count != count) return false;
    for (int i = 0; i < count; ++i)
        if (P->ctxs[i] != c[i] || P->uids[i] != c[i]->uid || P->versions[i] != c[i]->version ||
            P->fs[i] != f[i] || P->xs[i] != x[i])
            return false;
    return true;
}

template <class T, class TL>
static int solve_batched_ir(int count, mg_ctx *const *c, const double *const *f, double *const *x,
                            unsigned flags, mg_stats *st) {
    auto t0 = std::chrono::steady_clock::now();
    Ctx *c0 = c[0];
    BatchPlan *P = c0->plan;
    if (!plan_matches(P, count, c, f, x)) {
        batch_release(c0);
        P = new BatchPlan();
        c0->plan = P;
        P->count = count;
        P->st = c0->lp_store;
        for (int i = 0; i < count; ++i) {
            P->ctxs.push_back(c[i]);
            P->versions.push_back(c[i]->version);
            P->uids.push_back(c[i]->uid);
            P->fs.push_back(f[i]);
            P->xs.push_back(x[i]);
            P->xalt.push_back(c[i]->xalt);
        }
        if (hipStreamCreateWithFlags(&P->stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&P->ev_in, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&P->ev_out, hipEventDisableTiming) != hipSuccess ||
            hipMalloc(&P->flags, sizeof(int) * count) != hipSuccess ||
            hipMalloc(&P->partials, sizeof(double) * (size_t)count * kMaxRedBlocks * 2) != hipSuccess ||
            hipMalloc(&P->results, sizeof(double) * 4 * count) != hipSuccess ||
            hipHostMalloc((void **)&P->h_flags, sizeof(int) * count, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void **)&P->h_res, sizeof(double) * 4 * count, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void **)&P->h_one, sizeof(int), hipHostMallocDefault) != hipSuccess) {
            batch_release(c0);
            return set_err(MG_ENOMEM, "mg_solve_batched: allocation failed");
        }
        *P->h_one = 1;
        int rc = build_plan<T, TL>(P, count, c, f, x);
        if (rc != MG_OK) {
            batch_release(c0);
            return rc;
        }
    }
    hipStream_t s = P->stream;
    // order after the caller's stream
    BCK(hipEventRecord(P->ev_in, c0->stream));
    BCK(hipStreamWaitEvent(s, P->ev_in, 0));
    // initial pass: x := 0 (unless guesses are given), r = b - A x, ||r||, ||b||, flags
    BCK(fill_zero(s, P->flags, sizeof(int) * count));
    BCK(launch_ir<TL>(s, P->dbuf, P->ir_items[(flags & MG_GUESS) ? 3 : 2], P->ir_work, P->ir_nwork, P->count, false));
    BCK(hipMemcpyAsync(P->h_res, P->results, sizeof(double) * 4 * count, hipMemcpyDeviceToHost, s));
    BCK(hipStreamSynchronize(s));
    std::vector<double> bn(count), rel0(count), sc_used(count, 1.0);
    std::vector<int> fell(count, 0), conv_step(count, -1);
    bool refetch = false;
    for (int i = 0; i < count; ++i) {
        bn[i] = std::sqrt(P->h_res[4 * i + 1]);
        const double rn = std::sqrt(P->h_res[4 * i]);
        if (!std::isfinite(bn[i]) || !std::isfinite(rn))
            return set_err(MG_EINVAL, "mg_solve_batched: problem %d has a non-finite right-hand side or guess", i);
        if ((flags & MG_GUESS) && rn > bn[i]) {  // rejected guess: restart from zero
            BCK(fill_zero(s, x[i], c[i]->L[0].n * 8));
            fell[i] = 1;
            refetch = true;
        }
    }
    // Recompute the initial residuals where a guess was rejected (x is now
    // zero there) or where the residual must be scaled for its cast to the
    // inner storage type (the pass's final sum stored that scale; the
    // repeated pass uses it).  At most a few rounds: the residual changes
    // only where a guess was rejected.
    for (int round = 0; round < 3; ++round) {
        bool rescale = false;
        for (int i = 0; i < count; ++i)
            if (cast_scale(P->h_res[4 * i], (double)c[i]->L[0].n) != sc_used[i]) rescale = true;
        if (!refetch && !rescale) break;
        for (int i = 0; i < count; ++i) sc_used[i] = cast_scale(P->h_res[4 * i], (double)c[i]->L[0].n);
        BCK(launch_ir<TL>(s, P->dbuf, P->ir_items[(flags & MG_GUESS) ? 5 : 4], P->ir_work, P->ir_nwork, P->count,
                          false));
        BCK(hipMemcpyAsync(P->h_res, P->results, sizeof(double) * 4 * count, hipMemcpyDeviceToHost, s));
        BCK(hipStreamSynchronize(s));
        refetch = false;
    }
    int active = 0;
    for (int i = 0; i < count; ++i) {
        rel0[i] = bn[i] > 0.0 ? std::sqrt(P->h_res[4 * i]) / bn[i] : 0.0;
        if (bn[i] == 0.0 || rel0[i] <= c[i]->d.rtol) {
            conv_step[i] = 0;
            P->h_flags[i] = 1;
        } else {
            P->h_flags[i] = 0;
            ++active;
        }
    }
    BCK(hipMemcpyAsync(P->flags, P->h_flags, sizeof(int) * count, hipMemcpyHostToDevice, s));
    int max_cycles = 0;
    for (int i = 0; i < count; ++i) max_cycles = std::max(max_cycles, c[i]->d.max_cycles);
    // Each step: replay the graph, then read every problem's flag and
    // residual.  A problem whose residual diverges is stopped: its device
    // flag is set (from a pinned constant that the host never changes) so
    // that its work returns at once, and the call reports MG_EDIVERGED.
    std::vector<DivergenceWatch> watch(count);
    std::vector<int> diverged(count, 0);
    std::vector<double> rel_last(count, 0.0);
    int steps = 0;
    while (active > 0 && steps < max_cycles) {
        BCK(hipGraphLaunch(P->graph[steps & 1], s));
        BCK(hipMemcpyAsync(P->h_flags, P->flags, sizeof(int) * count, hipMemcpyDeviceToHost, s));
        BCK(hipMemcpyAsync(P->h_res, P->results, sizeof(double) * 4 * count, hipMemcpyDeviceToHost, s));
        BCK(hipStreamSynchronize(s));
        ++steps;
        active = 0;
        for (int i = 0; i < count; ++i) {
            if (conv_step[i] < 0 && !diverged[i]) {
                if (P->h_flags[i]) {
                    conv_step[i] = steps;
                } else {
                    const double rel = bn[i] > 0.0 ? std::sqrt(P->h_res[4 * i]) / bn[i] : 0.0;
                    rel_last[i] = rel;
                    if (watch[i].diverged(rel, rel0[i])) {
                        diverged[i] = steps;
                        BCK(hipMemcpyAsync(P->flags + i, P->h_one, sizeof(int), hipMemcpyHostToDevice, s));
                    }
                }
            }
            if (conv_step[i] < 0 && !diverged[i]) ++active;
        }
    }
    BCK(hipMemcpyAsync(P->h_res, P->results, sizeof(double) * 4 * count, hipMemcpyDeviceToHost, s));
    // iterates that stopped after an odd number of steps sit in the spare buffer
    for (int i = 0; i < count; ++i) {
        const int used = diverged[i] ? diverged[i] : (conv_step[i] < 0 ? steps : conv_step[i]);
        if (used & 1) BCK(hipMemcpyAsync(x[i], P->xalt[i], c[i]->L[0].n * 8, hipMemcpyDeviceToDevice, s));
    }
    BCK(hipStreamSynchronize(s));
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    int worst = MG_OK, first_div = -1;
    for (int i = 0; i < count; ++i) {
        mg_stats S{};
        S.cycles = diverged[i] ? diverged[i] : (conv_step[i] < 0 ? steps : conv_step[i]);
        S.rel_res0 = fell[i] ? 1.0 : rel0[i];
        S.rel_res = diverged[i] ? rel_last[i] : (bn[i] > 0.0 ? std::sqrt(P->h_res[4 * i]) / bn[i] : 0.0);
        S.fell_back = fell[i];
        S.ms = ms;
        if (conv_step[i] < 0) worst = MG_NOT_CONVERGED;
        if (diverged[i] && first_div < 0) first_div = i;
        if (st) st[i] = S;
    }
    if (first_div >= 0)
        return set_err(MG_EDIVERGED, "mg_solve_batched: the residual of problem %d diverged (%g after %d steps)",
                       first_div, rel_last[first_div], diverged[first_div]);
    return worst;
}

}  // namespace mg

using namespace mg;

extern "C" int mg_solve_batched(int count, mg_ctx *const *c, const double *const *f_dev,
                                double *const *x_dev, unsigned flags, mg_stats *st) {
    if (count < 0 || (count > 0 && (!c || !f_dev || !x_dev)))
        return set_err(MG_EINVAL, "mg_solve_batched: bad arguments");
    if (count == 0) return MG_OK;
    if (flags & ~(unsigned)MG_GUESS) return set_err(MG_EINVAL, "mg_solve_batched: unknown flags 0x%x", flags);
    for (int i = 0; i < count; ++i) {
        if (!c[i] || !f_dev[i] || !x_dev[i]) return set_err(MG_EINVAL, "mg_solve_batched: null entry %d", i);
        if (!c[i]->coeffs) return set_err(MG_EINVAL, "mg_solve_batched: problem %d has no coefficients", i);
        if (c[i]->has_diag)
            return set_err(MG_EINVAL, "mg_solve_batched: problem %d has a per-cell diagonal (single solves only)", i);
        if (c[i]->d.precision != c[0]->d.precision)
            return set_err(MG_EINVAL, "mg_solve_batched: problems must share one precision");
        if (c[i]->stream != c[0]->stream)
            return set_err(MG_EINVAL, "mg_solve_batched: problems must share one stream");
        for (int j = 0; j < i; ++j)
            if (c[j] == c[i]) return set_err(MG_EINVAL, "mg_solve_batched: context %d appears twice", i);
    }
    const int lp = c[0]->lp_store;
    if (lp < 0 || c[0]->d.nu1 < 1) {
        // FP64 V-cycles (or no pre-smoothing): the problems are solved one
        // after the other with the single-problem path
        int worst = MG_OK;
        for (int i = 0; i < count; ++i) {
            int rc = mg_solve(c[i], f_dev[i], x_dev[i], flags, st ? &st[i] : nullptr);
            if (rc < 0) return rc;
            worst = std::max(worst, rc);
        }
        return worst;
    }
    for (int i = 0; i < count; ++i)
        if (c[i]->d.nu1 != c[0]->d.nu1 || c[i]->d.nu2 != c[0]->d.nu2)
            return set_err(MG_EINVAL, "mg_solve_batched: problems must share nu1 and nu2");
    if (lp == ST_F32) return solve_batched_ir<float, float>(count, c, f_dev, x_dev, flags, st);
    return solve_batched_ir<bf16, bf16>(count, c, f_dev, x_dev, flags, st);
}
