// Batched solves (placeholder: sequential loop until the fused plan lands).
#include "mg_engine.h"

namespace mg {
void batch_release(Ctx *) {}
}  // namespace mg

extern "C" int mg_solve_batched(int count, mg_ctx *const *c, const double *const *f_dev,
                                double *const *x_dev, unsigned flags, mg_stats *st) {
    if (count < 0 || (count > 0 && (!c || !f_dev || !x_dev)))
        return mg::set_err(MG_EINVAL, "mg_solve_batched: bad arguments");
    int worst = MG_OK;
    for (int i = 0; i < count; ++i) {
        int rc = mg_solve(c[i], f_dev[i], x_dev[i], flags, st ? &st[i] : nullptr);
        if (rc < 0) return rc;
        if (rc > worst) worst = rc;
    }
    return worst;
}
