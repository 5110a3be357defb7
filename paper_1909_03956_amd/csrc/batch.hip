// Batched persistent prediction, graph capture and the autotuner.
#include "api_internal.h"

using namespace swv;

extern "C" {

int swv_batch_plan(swv_ctx, int, const swv_instance*, swv_plan* out) {
    if (out) *out = nullptr;
    return fail(SWV_ENOTSUP, "swv_batch_plan: not built yet");
}
int swv_plan_stats(swv_plan, swv_plan_stats_t*) { return fail(SWV_ENOTSUP, "not built yet"); }
int swv_batch_run(swv_plan) { return fail(SWV_ENOTSUP, "not built yet"); }
int swv_graph_capture(swv_plan, swv_graph* out) {
    if (out) *out = nullptr;
    return fail(SWV_ENOTSUP, "not built yet");
}
int swv_graph_launch(swv_graph) { return fail(SWV_ENOTSUP, "not built yet"); }
int swv_graph_destroy(swv_graph) { return SWV_OK; }
int swv_plan_destroy(swv_plan) { return SWV_OK; }
int swv_autotune(swv_ctx, const char*, int) { return fail(SWV_ENOTSUP, "not built yet"); }
int swv_tune_load(swv_ctx, const char*) { return fail(SWV_ENOTSUP, "not built yet"); }

}  // extern "C"
