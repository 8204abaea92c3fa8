// Library-internal: set the calling thread's keccak_last_error() message and
// return `code` (for translation units other than the one that owns it).
#pragma once

namespace kb {
int set_last_error(int code, const char* msg);
}  // namespace kb
