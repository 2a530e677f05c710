// Multilevel scaffold (placeholder until the coarsening kernels land).
#include "jet_internal.h"

extern "C" int jet_coarsen(jet_context *, const jet_csr *, const jet_params *, jet_hierarchy **, void *)
{
    return JET_ELIMIT;
}
extern "C" int jet_hierarchy_levels(const jet_hierarchy *) { return 0; }
extern "C" int jet_hierarchy_level(const jet_hierarchy *, int, jet_csr *, const int32_t **) { return JET_EINVAL; }
extern "C" void jet_hierarchy_free(jet_hierarchy *) {}
extern "C" int jet_partition(jet_context *, const jet_csr *, const jet_params *, int32_t *, jet_stats *, jet_trace *,
                             void *)
{
    return JET_ELIMIT;
}
