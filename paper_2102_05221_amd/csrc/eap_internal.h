// Library-internal interface between the C ABI (eap_api.cpp) and the request
// server (eap_serve.cpp).
#pragma once
#include <stddef.h>
#include <stdint.h>

#include "eap.h"

namespace eap {

// Sizes of a set of series whose offsets have already been checked.
struct SetSizes {
    int64_t n = 0, total = 0, maxlen = 0, minlen = 0;
};

// eap_nn1_workspace() for sets of these sizes, without re-reading offsets:
// the server sizes batch after batch against one candidate set.
size_t nn1_workspace_sizes(const SetSizes& Q, const SetSizes& R, const eap_params* p, const eap_nn_opts* o);

}  // namespace eap
