// state.h -- host-side services the step and run launchers share with the
// runtime: workspace buffers, instance lookup, error reporting.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/sevo.h"
#include "runtime.h"

namespace sevo {

// Library-owned device scratch, grown on demand and kept until the context
// is destroyed.  Calls on one context share it, so calls that overlap on
// different streams must not share a context.
enum { WS_PARTIAL = 0, WS_STEP = 1, WS_RUN = 2, WS_RUN_DESC = 3, WS_COUNT = 8 };
struct Workspace {
    struct Buf {
        void *ptr = nullptr;
        size_t bytes = 0;
    };
    Buf bufs[WS_COUNT];
    int get(sevo_ctx *ctx, int which, size_t bytes, void **out);
    void release();
};

struct InstanceView {
    const double *o;
    const double *M64;
    const float *Mfrag;
    const float *tab;
    const uint16_t *Mbf;
};

int set_error(sevo_ctx *ctx, int code, const char *msg);
int lookup_instance(sevo_ctx *ctx, const sevo_problem *p, uint32_t inst, InstanceView *out);
const Consts &ctx_consts(sevo_ctx *ctx);
uint32_t ctx_seed32(sevo_ctx *ctx);
Workspace &ctx_ws(sevo_ctx *ctx);
void release_state(sevo_ctx *ctx);

int eval_items(sevo_ctx *ctx, const std::vector<std::pair<EvalDesc, int>> &items, int precision,
               hipStream_t stream);
int eval_large(sevo_ctx *ctx, std::vector<EvalDesc> &v, bool bf16, hipStream_t stream);

}  // namespace sevo
