// Autotuner of the finest-level smoother tiles (placeholder).
#include "mg_engine.h"

extern "C" int mg_autotune(mg_ctx *c, int reps, int *tile, int *zchunk, double *us) {
    (void)reps;
    if (!c) return mg::set_err(MG_EINVAL, "mg_autotune: null context");
    if (tile) *tile = c->tile64;
    if (zchunk) *zchunk = c->zc64;
    if (us) *us = 0.0;
    return MG_OK;
}
