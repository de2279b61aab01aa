// Batched execution of many uneven Jacobi instances (placeholder until the
// persistent kernel lands).
#include "internal.h"

using namespace ao;

struct ao_batch {
    int dummy;
};

extern "C" {
int batch_create(const ao_args*, int, ao_batch**) { return fail(AO_ESTATE, "batched execution not available"); }
int batch_autotune(ao_batch*, void*, int, int, int*) { return fail(AO_ESTATE, "batched execution not available"); }
int batch_run(ao_batch*, void*, int) { return fail(AO_ESTATE, "batched execution not available"); }
int batch_info(const ao_batch*, int*, int*, int*) { return fail(AO_ESTATE, "batched execution not available"); }
int batch_destroy(ao_batch*) { return fail(AO_ESTATE, "batched execution not available"); }
}
