// Library-internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime_api.h>

#include "kbatch.h"

namespace kb {
// Set the calling thread's keccak_last_error() message and return `code`.
int set_last_error(int code, const char* msg);
// The captured graph of a kb_graph (owned by it), for embedding it as a
// child graph node.
hipGraph_t native_graph(kb_graph* g);
}  // namespace kb
