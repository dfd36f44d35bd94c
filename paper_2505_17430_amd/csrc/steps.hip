// steps.hip -- one-generation DE / PSO steps (unfused) and whole runs.
#include <hip/hip_runtime.h>

#include "../../include/sevo.h"
#include "runtime.h"
#include "state.h"

using namespace sevo;

void sevo::release_state(sevo_ctx *) {}

extern "C" {

int sevo_de_step(sevo_ctx *ctx, const sevo_problem *, uint32_t, const sevo_de_state *,
                 const sevo_de_params *, int32_t, void *)
{
    return set_error(ctx, SEVO_EUNSUPPORTED, "sevo_de_step: not built yet");
}

int sevo_pso_step(sevo_ctx *ctx, const sevo_problem *, uint32_t, const sevo_pso_state *,
                  const sevo_pso_params *, int32_t, void *)
{
    return set_error(ctx, SEVO_EUNSUPPORTED, "sevo_pso_step: not built yet");
}

int sevo_run(sevo_ctx *ctx, const sevo_run_desc *, int32_t, int32_t, sevo_run_result *, float *,
             int64_t, double *, int32_t, void *)
{
    return set_error(ctx, SEVO_EUNSUPPORTED, "sevo_run: not built yet");
}

}  // extern "C"
