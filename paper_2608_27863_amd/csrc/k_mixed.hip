// Mixed-precision condensation (FP32 factorisation with FP64-residual
// refinement).  Placeholder until the kernels land: reports "not supported".
#include <hip/hip_runtime.h>

#include "hdg_internal.h"

namespace hdg {

size_t condense_mixed_work_bytes(const hdg_ctx *ctx, int e0, int ne) {
    (void)ctx; (void)e0; (void)ne;
    return 256;
}

int launch_condense_mixed(const hdg_ctx *ctx, int e0, int ne, int refine, double *E, double *SK, int *info,
                          void *work, hipStream_t s) {
    (void)ctx; (void)e0; (void)ne; (void)refine; (void)E; (void)SK; (void)info; (void)work; (void)s;
    return (int)hipErrorNotSupported;
}

}  // namespace hdg
