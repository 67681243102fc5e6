// Batched path: many graphs in one persistent launch (work queue over (graph, vertex) items).
#include "internal.hpp"

namespace tcl {

void batch_engine_destroy(tc_lcc_ctx ctx) { (void)ctx; }

}  // namespace tcl

extern "C" tc_lcc_status tc_lcc_batch_submit(tc_lcc_ctx ctx, int count, const tc_lcc_graph* graphs,
                                             uint64_t* const* tri, double* const* lcc, tc_lcc_ticket* out) {
    (void)ctx; (void)count; (void)graphs; (void)tri; (void)lcc; (void)out;
    tcl::set_error("tc_lcc_batch_submit: not built yet");
    return TC_LCC_UNSUPPORTED;
}

extern "C" tc_lcc_status tc_lcc_batch_poll(tc_lcc_ctx ctx, tc_lcc_ticket t, int block, int* graphs_done) {
    (void)ctx; (void)t; (void)block; (void)graphs_done;
    tcl::set_error("tc_lcc_batch_poll: unknown ticket");
    return TC_LCC_INVALID_ARGUMENT;
}
