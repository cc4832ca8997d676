// Cost of the two ways of separating the phases of an iteration on one GPU,
// behind the choice of graph-replayed kernels over one persistent kernel for
// the uneven batch: a kernel boundary inside a captured HIP graph (mode 0:
// `rounds` launches of a kernel that touches one word per block, captured
// once and replayed), and a grid-wide barrier inside one cooperative kernel
// (mode 1: `rounds` grid barriers of a kernel with as many blocks as can be
// resident at once, launched with hipLaunchCooperativeKernel, which refuses a
// grid that could not be resident). Both use 256-thread blocks and the same
// per-round work.
#include <hip/hip_cooperative_groups.h>

#include "device.h"
#include "internal.h"

namespace petgem {

namespace {

namespace cg = cooperative_groups;

__global__ void __launch_bounds__(256) k_probe_round(int* __restrict__ w) {
    if (threadIdx.x == 0) w[blockIdx.x] += 1;
}

__global__ void __launch_bounds__(256) k_probe_persistent(int* __restrict__ w, int rounds) {
    cg::grid_group grid = cg::this_grid();
    for (int r = 0; r < rounds; ++r) {
        if (threadIdx.x == 0) w[blockIdx.x] += 1;
        grid.sync();
    }
}

}  // namespace

int sync_probe(int32_t rounds, int32_t mode, int32_t* blocks_out, float* us_per_round, hipStream_t s) {
    int dev = 0, ncu = 0, per_cu = 0;
    PG_HIP(hipGetDevice(&dev));
    PG_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    PG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k_probe_persistent),
                                                        256, 0));
    const int blocks = std::max(1, ncu * std::max(per_cu, 1));
    int* w = nullptr;
    PG_TRY(dalloc(&w, (size_t)blocks));
    PG_HIP(hipMemsetAsync(w, 0, sizeof(int) * (size_t)blocks, s));
    hipEvent_t e0, e1;
    PG_HIP(hipEventCreate(&e0));
    PG_HIP(hipEventCreate(&e1));
    int rc = PETGEM_OK;
    float ms = 0.f;
    if (mode == 0) {
        hipStream_t cs = nullptr;
        hipGraph_t g = nullptr;
        hipGraphExec_t ge = nullptr;
        PG_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        PG_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        for (int r = 0; r < rounds; ++r) hipLaunchKernelGGL(k_probe_round, dim3(blocks), dim3(256), 0, cs, w);
        PG_HIP(hipStreamEndCapture(cs, &g));
        PG_HIP(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
        PG_HIP(hipGraphLaunch(ge, s));   // warm-up
        PG_HIP(hipEventRecord(e0, s));
        PG_HIP(hipGraphLaunch(ge, s));
        PG_HIP(hipEventRecord(e1, s));
        PG_HIP(hipEventSynchronize(e1));
        PG_HIP(hipEventElapsedTime(&ms, e0, e1));
        (void)hipGraphExecDestroy(ge);
        (void)hipGraphDestroy(g);
        (void)hipStreamDestroy(cs);
    } else {
        int r_ = rounds;
        void* args[] = {&w, &r_};
        hipError_t e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_probe_persistent), dim3(blocks),
                                                  dim3(256), args, 0, s);   // warm-up
        if (e != hipSuccess) {
            set_error(std::string("cooperative launch: ") + hipGetErrorString(e));
            rc = PETGEM_HIP_ERROR;
        } else {
            PG_HIP(hipEventRecord(e0, s));
            PG_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_probe_persistent), dim3(blocks),
                                              dim3(256), args, 0, s));
            PG_HIP(hipEventRecord(e1, s));
            PG_HIP(hipEventSynchronize(e1));
            PG_HIP(hipEventElapsedTime(&ms, e0, e1));
        }
    }
    PG_HIP(hipStreamSynchronize(s));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    dfree(w);
    if (blocks_out) *blocks_out = blocks;
    if (us_per_round) *us_per_round = 1e3f * ms / (float)rounds;
    return rc;
}

}  // namespace petgem
