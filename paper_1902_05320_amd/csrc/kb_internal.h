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
// The autotuner's cache (tune_cache.cpp).  tune_lookup: the tile the cache at
// `path` (NULL: $KBATCH_TUNE) holds for a batch of n messages of `variant`
// (-1 = mixed) on the current device; 1 if found, 0 if not, < 0 on error.
int tune_lookup(const char* path, int variant, uint64_t n, kb_tile* out);
// Record the tile the calling thread's batch call runs (keccak_last_tile).
void note_tile(const kb_tile* t, int cached);
// Block-count class floor(log2(blocks)) capped at KB_NB_CLASSES - 1, and
// batch class floor(log2(n)).
int nb_class_of(uint64_t blocks);
int batch_class_of(uint64_t n);
}  // namespace kb
