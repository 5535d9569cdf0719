// MFMA precision form (placeholder until the kernels land).
#include "internal.h"

namespace csplat {

csplat_status precision_build(csplat_ctx *, csplat_scene *, uint32_t)
{
    return fail(CSPLAT_E_INVALID, "precision features are not available in this build");
}

csplat_status precision_eval(csplat_ctx *, const csplat_scene *, int64_t, const float *, const float *,
                             const EvalParams &, const EvalOut &, int)
{
    return fail(CSPLAT_E_INVALID, "precision forms are not available in this build");
}

}  // namespace csplat
