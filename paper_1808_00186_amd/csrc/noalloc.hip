// The allocation-free right-hand side (petgem_rhs_noalloc), for callers that
// cannot allocate device memory: code under HIP graph capture, tight serving
// loops, harnesses that forbid allocation. It runs the same kernels as
// petgem_rhs (Section 3, eq. 9 with the dipole field of Appendix A), but
// their scratch -- the singular-source flag and the element staging of six
// complex128 entries per element -- lives in one file-scope device array of
// fixed size instead of buffers the library allocates.
//
// Each GPU holds its own copy of the array, at its own address, until the
// process ends. The address is looked up once per device (with that device
// current) when a system is first assembled on it, or by the entry point's
// first call there; host code only ever passes that looked-up address, never
// the array's name. Every call on one GPU shares the array: the flag is
// cleared by a fill kernel at the start of each call, the staging is fully
// overwritten before it is read, and calls that overlap on one GPU (other
// streams, other threads) race.
#include <mutex>

#include "device.h"
#include "internal.h"

namespace petgem {

namespace {

constexpr int kNoAllocMaxTets = 1 << 19;     // 524,288 elements
constexpr size_t kFlagBytes = 256;          // the flag, padded to the array's alignment
constexpr size_t kScratchBytes = kFlagBytes + (size_t)6 * kNoAllocMaxTets * sizeof(double2);   // 48 MiB + 256 B
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

__global__ void k_clear_flag(int* f) {
    if (threadIdx.x == 0) f[0] = 0;
}

}  // namespace

// Address of this device's scratch array: looked up on the first call per
// device (the device must be current), then cached.
int noalloc_scratch(int dev, char** out) {
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device index out of range for the allocation-free scratch");
        return PETGEM_INVALID_ARG;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = -1;
        PG_HIP(hipGetDevice(&cur));
        if (cur != dev) {
            set_error("the allocation-free scratch is looked up with its device current");
            return PETGEM_INVALID_ARG;
        }
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            return PETGEM_HIP_ERROR;
        }
        g_scratch_ptr[dev] = static_cast<char*>(p);
    }
    *out = g_scratch_ptr[dev];
    return PETGEM_OK;
}

int rhs_noalloc(petgem_system* sys, const petgem_source* src, int32_t n_src, double2* b, hipStream_t s) {
    if (sys->n_tets > kNoAllocMaxTets) {
        set_error("petgem_rhs_noalloc: " + std::to_string(sys->n_tets) + " elements exceed its scratch of " +
                  std::to_string(kNoAllocMaxTets) + " elements; use petgem_rhs");
        return PETGEM_INVALID_ARG;
    }
    int cur = -1;
    PG_HIP(hipGetDevice(&cur));
    if (cur != sys->device) {
        set_error("petgem_rhs_noalloc: the system's device must be current");
        return PETGEM_INVALID_ARG;
    }
    char* base = nullptr;
    PG_TRY(noalloc_scratch(cur, &base));
    int* flag = reinterpret_cast<int*>(base);
    double2* Rst = reinterpret_cast<double2*>(base + kFlagBytes);
    hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(64), 0, s, flag);
    PG_HIP(hipGetLastError());
    for (int32_t k = 0; k < n_src; ++k)
        PG_TRY(launch_rhs_into(sys, src[k], b + (size_t)k * sys->n_dof, 1, Rst, flag, s));
    int flag_h = 0;
    PG_HIP(hipMemcpyAsync(&flag_h, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    if (flag_h) {
        set_error("source within 1e-9 h of a quadrature point of an element with dsigma != 0");
        return PETGEM_SOURCE_SINGULAR;
    }
    return PETGEM_OK;
}

}  // namespace petgem
