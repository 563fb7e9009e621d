// Batched execution of many independent problems (declared in dgsn.h).
#include "common.hpp"

using namespace dgsn;

extern "C" {

int dgsn_batch_create(dgsn_ctx *, dgsn_problem *const *, int, dgsn_batch **out)
{
    clear_error();
    if (out) *out = nullptr;
    return set_error(DGSN_EUNSUPPORTED, "batched execution is not available in this build");
}

int dgsn_batch_set_io(dgsn_batch *, int, const void *, void *)
{
    clear_error();
    return set_error(DGSN_EUNSUPPORTED, "batched execution is not available in this build");
}

int dgsn_batch_run(dgsn_batch *, void *)
{
    clear_error();
    return set_error(DGSN_EUNSUPPORTED, "batched execution is not available in this build");
}

int dgsn_batch_latencies_us(const dgsn_batch *, double *)
{
    clear_error();
    return set_error(DGSN_EUNSUPPORTED, "batched execution is not available in this build");
}

int dgsn_batch_destroy(dgsn_batch *)
{
    clear_error();
    return DGSN_OK;
}

}  // extern "C"
