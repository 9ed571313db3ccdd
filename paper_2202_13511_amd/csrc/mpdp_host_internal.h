// Host-side exact step for the large-query heuristics (mpdp_large.cpp):
// MPDP on a query whose relations are units (base relations or planned
// intermediate results, each with its plan's cost), one query at a time or
// many at once through the batched kernel.  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>

#include "mpdp.h"

namespace mpdp_host {

size_t units_workspace_bytes(uint32_t n);
size_t units_batch_workspace_bytes(uint32_t nq, const mpdp_batch_query *queries);

mpdp_status optimize_units(uint32_t n, uint32_t m, const mpdp_edge *edges, const double *card, const double *sel,
                           const double *base_costs, mpdp_cost_model cm, void *d_ws, size_t ws_bytes,
                           hipStream_t s, mpdp_plan_node *plan_out, double *cost_out);

mpdp_status optimize_units_batch(uint32_t nq, const mpdp_batch_query *queries, const mpdp_edge *edges,
                                 const double *card, const double *sel, const double *base_costs,
                                 mpdp_cost_model cm, void *d_ws, size_t ws_bytes, hipStream_t s,
                                 mpdp_plan_node *plans_out, double *costs_out);

// The no-allocation path (mpdp_noalloc.hip): the exact DP in a workspace
// the caller provides, with no host or device allocation in the call.
// noalloc_setup builds the host's static tables (call once before the first
// optimize_noalloc).  optimize_noalloc validates the query, then asks
// get_ws for the workspace (ws_bytes long); it returns MPDP_ETOOLARGE when
// that is too small for n relations.
size_t noalloc_workspace_bytes(uint32_t n);
const uint32_t *noalloc_setup();
mpdp_status optimize_noalloc(uint32_t n, uint32_t m, const mpdp_edge *edges, const double *card, const double *sel,
                             mpdp_cost_model cm, mpdp_status (*get_ws)(void **), size_t ws_bytes, hipStream_t s,
                             uint32_t flags, mpdp_plan_node *plan_out, double *cost_out, mpdp_stats *stats_out);

}  // namespace mpdp_host
