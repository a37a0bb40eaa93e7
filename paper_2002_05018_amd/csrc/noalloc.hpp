// Internal interface between the C ABI (d3m_api.cpp) and the allocation-free
// solve entry point (solve_noalloc.hip), which owns the static device scratch.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

struct d3m_problem;

namespace d3m {

// records msg as the calling thread's last error and returns code
int set_error(int code, const char *msg);
// HIP device ordinal of the handle
int handle_device(const d3m_problem *h);
// scratch bytes the FP64 solve of nrhs right-hand sides needs (D3M_ESTATE if
// the handle holds no FP64 factors)
int solve_scratch_bytes(const d3m_problem *h, int nrhs, size_t *bytes);
// the FP64 solve (recipe steps 6-7) with its vector arrays carved out of
// `scratch` (device memory of `bytes` bytes); kernel launches only, on s
int solve_into_scratch(d3m_problem *h, const double2 *f, double2 *E, int nrhs, void *scratch, size_t bytes,
                       hipStream_t s);

}  // namespace d3m
