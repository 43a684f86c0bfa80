// Internal C++ interface between the sort engine (ipls_lib.hip) and the request server
// (ipls_server.cpp).  An Engine is one context of cached device buffers; calls on one Engine are
// serialised, separate Engines run concurrently on their own streams.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/ipls.h"

namespace ipls {

struct Engine;

Engine* engine_new();
void engine_free(Engine* e);

// ipls_sort_ex on the given context.
ipls_status engine_sort(Engine& e, void* keys, uint32_t* payload, size_t n, ipls_dtype dtype, const ipls_params* p,
                        void* workspace, size_t workspace_bytes, ipls_stats* stats, hipStream_t s);

// ipls_sort_segmented on the given context, with an optional caller-owned workspace of
// ipls_workspace_bytes(total keys) bytes.
ipls_status engine_sort_segmented(Engine& e, void* keys, uint32_t* payload, const uint64_t* seg_offsets, size_t nseg,
                                  ipls_dtype dtype, const ipls_params* p, void* workspace, size_t workspace_bytes,
                                  ipls_stats* stats, hipStream_t s);

}  // namespace ipls
