// Autotuner of the finest-level smoother: every tile shape x z-chunk is
// timed with HIP events on the context's stream and the fastest is kept.
// Results are cached per (grid, storage type, coefficient mode) for the
// life of the process and, if the environment variable MG_TUNE_CACHE names
// a file, in that file (one "nx ny nz store mode tile zchunk us" line per
// entry).
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>

#include "mg_engine.h"

namespace mg {
namespace {

using Key = std::tuple<int, int, int, int, int>;
struct Val {
    int tile, zchunk;
    double us;
};

std::mutex g_tune_mu;
std::map<Key, Val> g_tune;
bool g_tune_loaded = false;

void load_cache_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = std::getenv("MG_TUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    int nx, ny, nz, st, mode, tile, zc;
    double us;
    while (std::fscanf(f, "%d %d %d %d %d %d %d %lf", &nx, &ny, &nz, &st, &mode, &tile, &zc, &us) == 8)
        if (tile >= 1 && tile <= kNumTiles && zc >= 1) g_tune[Key{nx, ny, nz, st, mode}] = Val{tile, zc, us};
    std::fclose(f);
}

void save_cache_locked() {
    const char *path = std::getenv("MG_TUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "w");
    if (!f) return;
    for (const auto &kv : g_tune) {
        const Key &k = kv.first;
        std::fprintf(f, "%d %d %d %d %d %d %d %.3f\n", std::get<0>(k), std::get<1>(k), std::get<2>(k),
                     std::get<3>(k), std::get<4>(k), kv.second.tile, kv.second.zchunk, kv.second.us);
    }
    std::fclose(f);
}

}  // namespace
}  // namespace mg

using namespace mg;

extern "C" int mg_autotune(mg_ctx *c, int reps, int *tile, int *zchunk, double *us) {
    if (!c) return set_err(MG_EINVAL, "mg_autotune: null context");
    if (!c->coeffs) return set_err(MG_EINVAL, "mg_autotune: mg_set_coeffs has not succeeded");
    if (reps < 1) reps = 1;
    const bool lowp = c->lp_store >= 0;
    const int st = lowp ? c->lp_store : ST_F64;
    if (c->tail == 0) {  // the whole grid is handled by the bottom solver: nothing to tune
        if (tile) *tile = 0;
        if (zchunk) *zchunk = 0;
        if (us) *us = 0.0;
        return MG_OK;
    }
    const Geo G = level_geo(c, 0, !lowp, lowp);
    const Coef C = level_coef(c, 0, lowp);
    const Key key{G.nx, G.ny, G.nz, st, C.mode};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        load_cache_locked();
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            if (lowp) { c->tile_lp = it->second.tile; c->zc_lp = it->second.zchunk; }
            else { c->tile64 = it->second.tile; c->zc64 = it->second.zchunk; }
            if (tile) *tile = it->second.tile;
            if (zchunk) *zchunk = it->second.zchunk;
            if (us) *us = it->second.us;
            return MG_OK;
        }
    }
    hipStream_t s = c->stream;
    const size_t bytes = c->L[0].n * store_size(st);
    void *a = nullptr, *b = nullptr;
    if (hipMalloc(&a, bytes) != hipSuccess) return set_err(MG_ENOMEM, "mg_autotune: allocation failed");
    if (hipMalloc(&b, bytes) != hipSuccess) {
        (void)hipFree(a);
        return set_err(MG_ENOMEM, "mg_autotune: allocation failed");
    }
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    int best_t = 0, best_z = 0;
    double best = 1e30;
    int rc = MG_OK;
    if (fill_zero(s, a, bytes) != hipSuccess) rc = MG_EDEVICE;
    const int zcands[] = {4, 8, 16, 32, 64, 128};
    for (int t = 1; t <= kNumTiles && rc == MG_OK; ++t) {
        for (int zc : zcands) {
            if (zc > G.nz && zc != zcands[0]) continue;
            // one warm-up launch, then reps timed launches
            if (smooth(s, st, G, C, a, b, a, false, t, zc) != hipSuccess) { rc = MG_EDEVICE; break; }
            if (hipEventRecord(e0, s) != hipSuccess) { rc = MG_EDEVICE; break; }
            for (int r = 0; r < reps; ++r)
                if (smooth(s, st, G, C, a, b, a, false, t, zc) != hipSuccess) { rc = MG_EDEVICE; break; }
            if (rc != MG_OK || hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                rc = MG_EDEVICE;
                break;
            }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            const double t_us = 1e3 * ms / reps;
            if (t_us < best) { best = t_us; best_t = t; best_z = zc; }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(a);
    (void)hipFree(b);
    if (rc != MG_OK) return set_err(rc, "mg_autotune: a timed launch failed");
    if (lowp) { c->tile_lp = best_t; c->zc_lp = best_z; }
    else { c->tile64 = best_t; c->zc64 = best_z; }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[key] = Val{best_t, best_z, best};
        save_cache_locked();
    }
    if (tile) *tile = best_t;
    if (zchunk) *zchunk = best_z;
    if (us) *us = best;
    return MG_OK;
}
