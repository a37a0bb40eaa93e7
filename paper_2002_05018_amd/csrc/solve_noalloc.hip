// d3m_solve_noalloc: the FP64 solve of d3m_solve for callers that cannot
// allocate device memory (code under HIP graph capture, serving loops, hosts
// that forbid allocation).  Its working vectors live in one file-scope device
// array; every GPU the library runs on holds its own copy until the process
// ends.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/d3m.h"
#include "noalloc.hpp"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // D3M_NOALLOC_SCRATCH_BYTES
static_assert(kScratchBytes == (size_t)D3M_NOALLOC_SCRATCH_BYTES, "header and array disagree");

// Device-side storage.  In host code this name is only a stand-in for the
// symbol: the device address comes from hipGetSymbolAddress (per device).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// Address of this device's copy of the array, looked up once per device with
// that device current.
int scratch_ptr(int dev, void **out) {
    if (dev < 0 || dev >= kMaxDevices) return d3m::set_error(D3M_ENODEV, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return d3m::set_error(D3M_EHIP, (std::string("hipGetSymbolAddress of the solve scratch: ") +
                                             hipGetErrorString(e)).c_str());
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return D3M_OK;
}

bool on_device(const void *p) {
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice;
}

}  // namespace

extern "C" int d3m_solve_noalloc(d3m_handle h, const d3m_c128 *rhs, int32_t nrhs, d3m_c128 *E, void *stream) {
    if (!h || !rhs || !E) return d3m::set_error(D3M_EINVAL, "null argument");
    if (nrhs < 1) return d3m::set_error(D3M_EINVAL, "nrhs must be >= 1");
    const int dev = d3m::handle_device(h);
    if (hipSetDevice(dev) != hipSuccess) return d3m::set_error(D3M_EHIP, "hipSetDevice failed");
    size_t need = 0;
    int rc = d3m::solve_scratch_bytes(h, nrhs, &need);
    if (rc != D3M_OK) return rc;
    if (need > kScratchBytes) {
        const std::string msg = "the allocation-free solve needs " + std::to_string(need) +
                                " bytes of scratch for " + std::to_string(nrhs) +
                                " right-hand sides; its limit is " + std::to_string(kScratchBytes) +
                                " (use d3m_solve, or fewer right-hand sides per call)";
        return d3m::set_error(D3M_EINVAL, msg.c_str());
    }
    if (!on_device(rhs) || !on_device(E))
        return d3m::set_error(D3M_EINVAL, "the allocation-free solve takes device buffers only");
    void *p = nullptr;
    if ((rc = scratch_ptr(dev, &p)) != D3M_OK) return rc;
    return d3m::solve_into_scratch(h, reinterpret_cast<const double2 *>(rhs), reinterpret_cast<double2 *>(E), nrhs,
                                   p, kScratchBytes, (hipStream_t)stream);
}
