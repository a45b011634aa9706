// Fused single-launch forward + contraction + adjoint path (under construction).
#include "internal.h"

namespace vp {

vpinn_status fused_loss_grad(vpinn_problem *, const vpinn_loss_cfg *, const float *, const float *, float *, float *,
                             float *, hipStream_t) {
    return fail(VPINN_E_UNSUPPORTED, "the fused path is not available in this build");
}

}  // namespace vp
