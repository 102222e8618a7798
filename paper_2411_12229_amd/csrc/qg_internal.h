// qg_internal.h -- pieces of the index shared by the host-side parts of libqg
// (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "qg.h"

namespace qgi {

// A second handle on an index: it shares the rotation and the vertex blocks
// (which stay owned by `base`) but has its own scratch, counters and stream, so
// searches through different views may run concurrently.  Freed with
// qg_free_index; `base` must outlive it.  nullptr on failure (qg_last_error).
qg_index* make_view(const qg_index* base);

// Sets the thread's qg_last_error message and returns `code`.
int set_error(int code, const std::string& msg);

int device_of(const qg_index* idx);
int dim_of(const qg_index* idx);

}  // namespace qgi
