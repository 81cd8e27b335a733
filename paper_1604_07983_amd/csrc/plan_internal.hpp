// plan_internal.hpp -- plan functions shared by the C ABI's source files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "../../include/nbs.h"

namespace nbs {

// nbs_plan_create with an optional device workspace: when arena is given the
// plan carves every device buffer from [arena, arena + arena_size) instead
// of allocating (NBS_ERR_UNSUPPORTED when it does not fit), uploads its
// tables on upload_stream and waits for them, and nbs_plan_destroy frees
// only host memory.
nbs_status create_plan(nbs_plan* out, const nbs_geometry* g, int32_t n_geom, const nbs_channel* ch, int32_t n_ch,
                       nbs_precision prec, int32_t device, void* arena, size_t arena_size, hipStream_t upload_stream);

// Enqueue build, contraction and relative sum on st.
nbs_status run_plan(nbs_plan p, const void* const* pu, const void* const* pd, const void* const* ps,
                    void* const* F_out, hipStream_t st);

const char* plan_error(const nbs_plan p);
// Why the calling thread's last create_plan failed ("" if it did not say).
const char* create_error();

}  // namespace nbs
