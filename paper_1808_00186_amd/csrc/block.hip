// Multi-source COCG and the uneven multi-system batch (mixed precision).
#include "device.h"
#include "internal.h"

namespace petgem {

struct BlockWork {
    int dummy = 0;
};

void release_block_work(BlockWork*& w) {
    delete w;
    w = nullptr;
}

int block_solve(petgem_system*, const petgem_source*, int32_t, const petgem_opts&, const double2*,
                double2*, hipStream_t, petgem_stats*) {
    set_error("COCG path not built");
    return PETGEM_INVALID_ARG;
}

int batch_solve(petgem_system* const*, const petgem_source*, int32_t, const petgem_opts&,
                petgem_solution**, hipStream_t, petgem_stats*) {
    set_error("batch path not built");
    return PETGEM_INVALID_ARG;
}

}  // namespace petgem
