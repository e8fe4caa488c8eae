// Internal entry points shared by the C ABI and the request server: the same
// operations as pne_network_create / pne_batch_create, enqueued on a given
// stream instead of the context's.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "pne.h"

namespace pne {

pne_status network_create_on(pne_ctx *ctx, const pne_network_desc *desc, int on_device, hipStream_t stream,
                             pne_network **out);
// A device region a batch places all its tables and buffers in instead of
// allocating (the allocation-free entry point).
struct StaticArena {
    char *base = nullptr;
    size_t cap = 0;
};

// fixed != nullptr: no device or pinned allocation, no events; the batch
// allows one outstanding launch, and the flags PROFILE, GRAPH and AUTOTUNE
// are refused.
pne_status batch_create_on(pne_ctx *ctx, pne_network *const *nets, int32_t n, const pne_options *opt,
                           hipStream_t stream, pne_batch **out, const StaticArena *fixed = nullptr);

// Context access for the other entry points (strip expansions).
hipStream_t ctx_stream(pne_ctx *ctx);
int ctx_device(pne_ctx *ctx);
// Network access for the other entry points: site count, graph (false when
// the network has open legs), per-site device tensor, geometry equality.
int network_sites(pne_network *net);
bool network_graph(pne_network *net, std::vector<int> *rank, std::vector<int> *bond_dims, std::vector<int> *bu,
                   std::vector<int> *bul, std::vector<int> *bv, std::vector<int> *bvl);
const double *network_site_ptr(pne_network *net, int site);
bool same_geometry(pne_network *a, pne_network *b);
// Record msg as the context's last error and return st.
pne_status ctx_fail(pne_ctx *ctx, pne_status st, const std::string &msg);

}  // namespace pne
