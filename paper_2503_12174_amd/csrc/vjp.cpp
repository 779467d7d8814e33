// vjp.cpp -- dpcs_render_vjp orchestration (entry point; adjoint kernels follow).
#include "runtime.hpp"

extern "C" dpcs_status dpcs_render_vjp(dpcs_context ctx, dpcs_scene, const dpcs_render_params*, const float*,
                                       const float*, const float*, const dpcs_grads*) {
    return dpcs::fail(ctx, DPCS_E_UNSUPPORTED, "VJP not available in this build");
}
