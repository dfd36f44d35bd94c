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
enum { WS_PARTIAL = 0, WS_STEP = 1, WS_RUN = 2, WS_RUN_DESC = 3, WS_CSO = 4, WS_OPERANDS = 5, WS_COUNT = 8 };
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

// One kernel launch of a call, kept by a plan (sevo_plan_*) to be enqueued
// again later with nothing but launches.
enum { L_SMALL = 0, L_F64 = 1, L_LARGE = 2, L_COMBINE = 3, L_RUN = 4, L_CSO = 5, L_OPERANDS = 6 };
struct Launch {
    int kind;
    const void *d;      // device descriptors
    int n, ks, total, grid;   // ks: L_SMALL K steps; L_LARGE points per workgroup
    bool flag;          // L_SMALL, L_LARGE, L_OPERANDS: split bf16; L_RUN: population on chip
    bool wave;          // L_RUN: wave teams
    size_t shm;         // L_RUN: dynamic LDS bytes
    int stride;         // L_RUN: floats of dynamic LDS per run
    int lane;           // internal stream of the launch (runs: one per group)
    int fam = 0;        // L_RUN: algorithm family (kernel family of the runs)
};
// While a plan is being built the context records launches instead of
// enqueueing them, and descriptor tables and workspace come from
// plan-owned device memory (ctx_recording() != nullptr).
sevo_plan *ctx_recording(sevo_ctx *ctx);
int emit_launch(sevo_ctx *ctx, const Launch &L, hipStream_t stream);
int plan_alloc(sevo_ctx *ctx, size_t bytes, void **out);
hipError_t exec_run_launch(const Launch &L, hipStream_t stream, uint32_t seed32, const Consts &k);
// Start recording a plan on the context; plan_finish stops, and on success
// (rc == 0) hands the plan out, else frees it and returns rc.
int plan_begin(sevo_ctx *ctx);
int plan_finish(sevo_ctx *ctx, int rc, sevo_plan **out);

// Makes the context's GPU current for the scope of a call.
struct DeviceScope {
    int prev = -1;
    explicit DeviceScope(sevo_ctx *ctx);
    ~DeviceScope();
};

// Stage bytes in device memory on `stream` (content-cached, see runtime.hip);
// finish_slot records that the kernels reading the slot are queued.
int stage_blob(sevo_ctx *ctx, const std::vector<char> &blob, hipStream_t stream, const void **d_out,
               int *slot_out);
int finish_slot(sevo_ctx *ctx, int slot, hipStream_t stream);

// Fork `n` internal streams off `parent` (each waits for the work queued on
// parent so far) and join them back (parent waits for all of them).
int fork_streams(sevo_ctx *ctx, hipStream_t parent, int n, hipStream_t *out);
int join_streams(sevo_ctx *ctx, hipStream_t parent, int n, const hipStream_t *streams);
int lookup_instance(sevo_ctx *ctx, const sevo_problem *p, uint32_t inst, InstanceView *out);
const Consts &ctx_consts(sevo_ctx *ctx);
uint32_t ctx_seed32(sevo_ctx *ctx);
Workspace &ctx_ws(sevo_ctx *ctx);
void release_state(sevo_ctx *ctx);

int eval_items(sevo_ctx *ctx, const std::vector<std::pair<EvalDesc, int>> &items, int precision,
               hipStream_t stream);
// The launches of one evaluation with their descriptor tables, not yet
// staged: L.d is filled in by whoever uploads `table`.  Large-D items take
// their partial sums from `part` (large_partial_floats floats) and their
// GEMM operands from `opnd` (large_operand_bytes bytes).
struct PreparedLaunch {
    Launch L;
    std::vector<char> table;
};
size_t large_partial_floats(const std::vector<EvalDesc> &items, int precision);
size_t large_operand_bytes(const std::vector<EvalDesc> &items, int precision);
int prepare_eval(sevo_ctx *ctx, std::vector<EvalDesc> items, int precision, float *part, void *opnd,
                 std::vector<PreparedLaunch> &out);

// CSO runs (cso.hip): a loop of update kernels and batched evaluations.
int cso_runs(sevo_ctx *ctx, const sevo_run_desc *runs, int n, int precision, sevo_run_result *results,
             float *trace, int64_t trace_len, double *best_x, int max_dim, hipStream_t stream);
hipError_t exec_cso_launch(const Launch &L, hipStream_t stream, uint32_t seed32, const Consts &k);

// Plain double-precision runs (steps.hip): one run at a time, one launch per
// generation step.
int run_plain_f64(sevo_ctx *ctx, const sevo_run_desc *runs, int n, sevo_run_result *results,
                  float *trace, int64_t trace_len, double *best_x, int max_dim, hipStream_t stream);

}  // namespace sevo
