// Internal declarations of the HIP library: the system and solution handles,
// device-side helpers and the kernel launchers shared by the .hip units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/petgem.h"
#include "mesh.h"

namespace petgem {

constexpr double kPi = 3.14159265358979323846;
constexpr double kMu0 = 4.0e-7 * kPi;
constexpr int kMaxRestart = 64;

void set_error(const std::string& msg);

// ---------------------------------------------------------------- errors
#define PG_HIP(call)                                                          \
    do {                                                                      \
        hipError_t e_ = (call);                                               \
        if (e_ != hipSuccess) {                                               \
            ::petgem::set_error(std::string(#call) + ": " + hipGetErrorString(e_)); \
            return e_ == hipErrorOutOfMemory ? PETGEM_OUT_OF_MEMORY : PETGEM_HIP_ERROR; \
        }                                                                     \
    } while (0)

#define PG_TRY(call)                      \
    do {                                  \
        int rc_ = (call);                 \
        if (rc_ != PETGEM_OK) return rc_; \
    } while (0)

template <class T>
inline int dalloc(T** p, size_t count) {
    *p = nullptr;
    if (count == 0) return PETGEM_OK;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T));
    if (e != hipSuccess) {
        set_error(std::string("hipMalloc of ") + std::to_string(count * sizeof(T)) + " bytes: " +
                  hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? PETGEM_OUT_OF_MEMORY : PETGEM_HIP_ERROR;
    }
    return PETGEM_OK;
}
template <class T>
inline void dfree(T*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

// Sliced-ELLPACK copy of the complex64 operator (the pattern and the real K,
// M_sigma values): slices of 64 rows, stored column-major inside a slice so a
// wavefront reads one entry of each of its 64 rows per load; rows are padded
// to the slice's longest with zero values that point at the row itself.
// Inside every 256-row tile the rows are ordered by length (longest first,
// then by index) before they are cut into slices, so that a slice holds rows
// of like length: on a 434k-DOF marine mesh this takes the padding from 18.6 % of the
// nonzeros to 6.7 %. row[] maps each slice lane back to its matrix row.
struct Sell {
    int nsl = 0;
    int64_t elems = 0;
    int32_t* ptr = nullptr;   // [nsl + 1] first element of each slice
    int32_t* w = nullptr;     // [nsl] slice width
    int32_t* row = nullptr;   // [nsl * 64] matrix row of each slice lane
    int32_t* col = nullptr;   // [elems]
    float* K = nullptr;       // [elems]
    float* M = nullptr;       // [elems]
    bool values = false;      // K, M current
    void release() {
        dfree(ptr); dfree(w); dfree(row); dfree(col); dfree(K); dfree(M);
        nsl = 0;
        elems = 0;
        values = false;
    }
};

// Multicolour split of the complex64 operator for the SSOR preconditioner:
// the DOFs coloured so that no two of a colour share a matrix entry, rows
// listed colour by colour (in DOF order within a colour), and for each listed
// row its entries coupling to earlier colours (L) and to later colours (U),
// the diagonal left out. pos: the entry's position in the CSR arrays, from
// which the values are gathered again whenever K32, Ms32 change.
struct Ssor {
    int nc = 0;                        // colours
    std::vector<int32_t> cptr;         // host [nc + 1] listed rows of each colour
    std::vector<int32_t> color_h;      // host [n] colour of each DOF
    int32_t* row = nullptr;            // [n] DOF of each listed row
    int32_t *lrp = nullptr, *lcol = nullptr, *lpos = nullptr;   // [n + 1], [nl], [nl]
    int32_t *urp = nullptr, *ucol = nullptr, *upos = nullptr;   // [n + 1], [nu], [nu]
    float *lK = nullptr, *lM = nullptr, *uK = nullptr, *uM = nullptr;
    double2* dg = nullptr;             // [n] {Kd, Md} of each listed row (read contiguously by the sweeps)
    int64_t nl = 0, nu = 0;
    bool values = false;               // lK .. uM, dg current
    void release() {
        dfree(row); dfree(lrp); dfree(lcol); dfree(lpos); dfree(urp); dfree(ucol); dfree(upos);
        dfree(lK); dfree(lM); dfree(uK); dfree(uM); dfree(dg);
        nc = 0; nl = nu = 0; values = false;
        cptr.clear(); color_h.clear();
    }
};

// Background of the primary field: the whole space sigma_bg, or two
// half-spaces meeting at z = z0 (s_up above, holding the sources).
struct Layers {
    int on = 0;
    double z0 = 0.0, s_up = 1.0, s_dn = 1.0;
};

// ------------------------------------------------------- GMRES control block
// Small device-resident state of one GMRES cycle: the Hessenberg column in
// progress, Givens rotations, the least-squares right-hand side g and flags
// that let every later kernel of the cycle exit early once it has converged.
struct GmresCtl {
    double2 H[(kMaxRestart + 1) * kMaxRestart];  // column-major, ld = kMaxRestart+1
    double2 cs[kMaxRestart], sn[kMaxRestart];
    double2 g[kMaxRestart + 1];
    double2 h[kMaxRestart + 1];                   // coefficients of the current pass
    double2 y[kMaxRestart];
    double nrm2;        // |w|^2 of the current pass
    double scale;       // multiplier applied by the update kernel
    double tol_abs;     // rtol * |b|
    double rnorm;       // true residual norm at the start of the cycle
    int done;           // cycle finished (converged estimate or breakdown)
    int reorth;         // second Gram-Schmidt pass requested
    int mdone;          // Arnoldi steps completed in this cycle
    int nonfinite;
};

struct GmresWork {
    int n = 0, m = 0, nb_dot = 0;
    double2* V = nullptr;        // (m+1) x n basis
    double2* u = nullptr;        // scaled iterate D x
    double2* b = nullptr;        // right-hand side of the current source
    double* partial = nullptr;   // [(m+2)][nb_dot] complex partial sums
    GmresCtl* ctl = nullptr;
    GmresCtl* ctl_host = nullptr;  // pinned mirror for the per-cycle readback
    hipGraphExec_t graph = nullptr;  // one captured cycle
    hipStream_t graph_stream = nullptr;
    void release();
};

// ------------------------------------------------------- multi-RHS workspace
struct BlockWork;   // defined in block.hip
void release_block_work(BlockWork*& w);

struct ReceiverCache {
    std::vector<double> rx;     // host copy of the located coordinates
    int32_t n_rx = 0;
    int32_t* tet = nullptr;     // device [n_rx]
    int32_t* dof = nullptr;     // device [n_rx][6]
    double* xyz = nullptr;      // device [n_rx][3]
    void release() { dfree(tet); dfree(dof); dfree(xyz); n_rx = 0; rx.clear(); }
};

}  // namespace petgem

struct petgem_system {
    int device = 0;
    int32_t n_nodes = 0, n_tets = 0, n_dof = 0, n_edges = 0;
    int64_t nnz = 0;
    double h_mean = 0.0;
    double sigma_bg = 1.0;
    petgem::Layers layers;                // layered background (layers.on) of the primary field
    double setup_seconds = 0.0;
    // host copies kept for receivers and accessors
    std::vector<double> xyz_h;
    std::vector<int32_t> tets_h;
    std::vector<int32_t> elem_dof_h;      // [T][6] DOF or -1
    std::vector<int32_t> dof_nodes_h;     // [n_dof][2]
    std::vector<int32_t> row_ptr_h;       // kept for host-side tools
    // device topology
    double* xyz = nullptr;                // [N][3]
    int32_t* tets = nullptr;              // [T][4]
    double* sigma = nullptr;              // [T]
    int32_t* row_ptr = nullptr;           // [n+1]
    int32_t* col = nullptr;               // [nnz]
    int32_t* diag_pos = nullptr;          // [n]
    int32_t* cptr = nullptr;              // [nnz+1]
    int32_t* cidx = nullptr;              // contributions
    int32_t* iptr = nullptr;              // [n+1]
    int32_t* islot = nullptr;             // incidence slots
    // assembled real matrices (frequency independent)
    double* Kst = nullptr;                // [21][T] staging
    double* Mst = nullptr;                // [21][T] staging (sigma-weighted)
    double* K = nullptr;                  // [nnz]
    double* Ms = nullptr;                 // [nnz]
    double* Kd = nullptr;                 // [n]
    double* Msd = nullptr;                // [n]
    // single-precision copies for the mixed-precision path
    float* K32 = nullptr;
    float* Ms32 = nullptr;
    bool have32 = false;
    petgem::Sell sell32;     // sliced-ELLPACK copy of K32 / Ms32 (built on first use)
    petgem::Ssor ssor32;     // multicolour L / U split of K32 / Ms32 (built on first SSOR use)
    // frequency-specific operator of the FP64 GMRES: Ahat = A D^{-1}
    double cached_freq = -1.0;
    double2* Ahat = nullptr;              // [nnz]
    double2* dvec = nullptr;              // [n] D = diag(A)
    double2* dinv = nullptr;              // [n]
    // right-hand-side staging and error flag
    double2* Rst = nullptr;               // [6][T]
    int* dflag = nullptr;                 // device error flags
    double2* tmp = nullptr;               // [n] scratch of petgem_spmv
    // voxel grid of the learned initial guess (cached at first use)
    int32_t* vox_tet = nullptr;           // [32^3] element containing each voxel centre
    int32_t* vox_dof = nullptr;           // [32^3][6]
    double* dof_mid = nullptr;            // [n][3] edge midpoints
    double* dof_tan = nullptr;            // [n][3] unit tangents (lo -> hi)
    double vox_lo[3] = {0.0, 0.0, 0.0};
    double vox_h = 0.0, vox_L = 0.0;
    int spmv_group = 8;                   // lanes per CSR row (autotuned)
    bool spmv_tuned = false;
    float spmv_tune_ms[3] = {0.f, 0.f, 0.f};  // measured 4/8/16-lane SpMV times
    petgem::GmresWork gw;
    petgem::BlockWork* bw = nullptr;
    petgem::ReceiverCache rxc;
};

struct petgem_solution {
    petgem_system* sys = nullptr;
    int32_t n_src = 0;
    double2* x = nullptr;                 // [n_src][n_dof]
    std::vector<petgem_source> src;
    double sigma_bg = 1.0;
    petgem::Layers layers;                // the background the solve used
};

namespace petgem {

// Launchers implemented in the .hip units; all ordered on `s`.
int launch_assembly(petgem_system* sys, hipStream_t s);
int launch_freq_prep(petgem_system* sys, double freq, hipStream_t s);
// allocation-free scratch of this device (looked up once per device) and the
// right-hand side that uses it
int noalloc_scratch(int dev, char** out);
int rhs_noalloc(petgem_system* sys, const petgem_source* src, int32_t n_src, double2* b, hipStream_t s);
int launch_rhs_into(petgem_system* sys, const petgem_source& src, double2* b, int b_stride, double2* Rst,
                    int* flag, hipStream_t s);
// time per round of a graph-replayed kernel boundary (mode 0) or of a grid
// barrier in one cooperative kernel (mode 1), probe.hip
int sync_probe(int32_t rounds, int32_t mode, int32_t* blocks_out, float* us_per_round, hipStream_t s);
// layered background (layered.hip)
int launch_rhs_layered(petgem_system* sys, const petgem_source& src, double2* Rst, int* flag, hipStream_t s);
int launch_receivers_layered(const petgem_solution* sol, int k, int32_t n_rx, double2* E, double2* Es,
                             hipStream_t s);
int launch_rhs(petgem_system* sys, const petgem_source& src, double2* b, int b_stride,
               hipStream_t s);
int launch_spmv_ahat(petgem_system* sys, const double2* x, double2* y, hipStream_t s);
int tune_spmv(petgem_system* sys, hipStream_t s);
int launch_spmv_unscaled(petgem_system* sys, const double2* x, double2* y, hipStream_t s);
int launch_receivers(const petgem_solution* sol, int32_t n_rx, double2* E, double2* Es,
                     hipStream_t s, bool magnetic = false);
int gmres_solve(petgem_system* sys, const petgem_source& src, const petgem_opts& o,
                const double2* x0, double2* x_out, hipStream_t s, petgem_stats* st);
int block_solve(petgem_system* sys, const petgem_source* src, int32_t n_src,
                const petgem_opts& o, const double2* x0, double2* x_out, hipStream_t s,
                petgem_stats* st);
int batch_solve(petgem_system* const* systems, const petgem_source* src, int32_t n_sys,
                const petgem_opts& o, const void* const* x0, petgem_solution** sols, hipStream_t s,
                petgem_stats* st);
int ensure_fp32(petgem_system* sys, hipStream_t s);
// the multicolour split of the operator (pattern built once, values gathered
// again after every reassembly); ssor_apply: z = M^-1 r of one complex64
// column at one frequency (device vectors of n_dof)
int ensure_ssor(petgem_system* sys, hipStream_t s);
int ssor_apply1(petgem_system* sys, double freq, double omega, const float2* r, float2* z, hipStream_t s);
// complex64 SpMM shapes the autotuner times for C columns (codes as the
// spmv_shape statistic); returns the count, writes at most cap codes
int spmm_candidate_codes(int C, bool sliced, int32_t* out, int cap);

// Grid helpers
inline int ceil_div(int64_t a, int64_t b) { return int((a + b - 1) / b); }

}  // namespace petgem
