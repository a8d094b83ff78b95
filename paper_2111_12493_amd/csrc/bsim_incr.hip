// bsim_incr.hip -- incremental summarization (resident state, update batches).
#include "bsim_api_internal.h"

namespace bsim {

int summarize_with_state(bsim_ctx* ctx, const bsim_graph&, const bsim_params&, bsim_state**,
                         bsim_result**) {
    ctx->err = "incremental state not available in this build";
    return BSIM_E_UNSUPPORTED;
}

}  // namespace bsim

extern "C" {

int bsim_apply_updates(bsim_state*, const bsim_update*, uint64_t, bsim_result** out) {
    if (out) *out = nullptr;
    return BSIM_E_UNSUPPORTED;
}

int bsim_state_graph(const bsim_state*, bsim_graph*) { return BSIM_E_UNSUPPORTED; }

void bsim_state_free(bsim_state*) {}

int bsim_batch_summarize(bsim_ctx*, const bsim_graph*, uint32_t, const bsim_params*, bsim_result** outs) {
    (void)outs;
    return BSIM_E_UNSUPPORTED;
}

}  // extern "C"
