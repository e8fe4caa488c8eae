// Internal entry points shared by the C ABI and the request server: the same
// operations as pne_network_create / pne_batch_create, enqueued on a given
// stream instead of the context's.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "pne.h"

namespace pne {

pne_status network_create_on(pne_ctx *ctx, const pne_network_desc *desc, int on_device, hipStream_t stream,
                             pne_network **out);
pne_status batch_create_on(pne_ctx *ctx, pne_network *const *nets, int32_t n, const pne_options *opt,
                           hipStream_t stream, pne_batch **out);

// Context access for the other entry points (strip expansions).
hipStream_t ctx_stream(pne_ctx *ctx);
int ctx_device(pne_ctx *ctx);
// Record msg as the context's last error and return st.
pne_status ctx_fail(pne_ctx *ctx, pne_status st, const std::string &msg);

}  // namespace pne
