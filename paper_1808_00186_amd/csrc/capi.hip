// The C ABI (include/petgem.h): argument checks, handle lifetime, host
// preprocessing and upload, and dispatch to the GPU stages.
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "device.h"
#include "internal.h"

namespace petgem {

namespace {
thread_local std::string g_err;

// complex entries (DOF x sources) from which a multi-frequency COCG block is
// solved one frequency run at a time
constexpr int64_t kFreqRunMin = 100000000;

int check_sys(const petgem_system* sys) {
    if (!sys) {
        set_error("null system handle");
        return PETGEM_INVALID_ARG;
    }
    return PETGEM_OK;
}

int valid_source(const petgem_source& s) {
    const double dn = std::sqrt(s.dir[0] * s.dir[0] + s.dir[1] * s.dir[1] + s.dir[2] * s.dir[2]);
    if (!(s.freq_hz > 0.0) || !std::isfinite(s.freq_hz) || !(std::fabs(dn - 1.0) < 1e-6) ||
        !std::isfinite(s.moment) || !std::isfinite(s.pos[0]) || !std::isfinite(s.pos[1]) ||
        !std::isfinite(s.pos[2])) {
        set_error("invalid source: frequency must be > 0, direction a unit vector, values finite");
        return PETGEM_INVALID_ARG;
    }
    return PETGEM_OK;
}

int upload_topology(petgem_system* sys, const HostTopology& t, const double* sigma, hipStream_t s) {
    const int64_t T = t.n_tets, n = t.n_dof;
    PG_TRY(dalloc(&sys->xyz, 3 * (size_t)t.n_nodes));
    PG_TRY(dalloc(&sys->tets, 4 * (size_t)T));
    PG_TRY(dalloc(&sys->sigma, (size_t)T));
    PG_TRY(dalloc(&sys->row_ptr, (size_t)n + 1));
    PG_TRY(dalloc(&sys->col, (size_t)t.nnz));
    PG_TRY(dalloc(&sys->diag_pos, (size_t)n));
    PG_TRY(dalloc(&sys->cptr, (size_t)t.nnz + 1));
    PG_TRY(dalloc(&sys->cidx, t.contrib_idx.size()));
    PG_TRY(dalloc(&sys->iptr, (size_t)n + 1));
    PG_TRY(dalloc(&sys->islot, t.inc_slot.size()));
    PG_TRY(dalloc(&sys->Kst, 21 * (size_t)T));
    PG_TRY(dalloc(&sys->Mst, 21 * (size_t)T));
    PG_TRY(dalloc(&sys->K, (size_t)t.nnz));
    PG_TRY(dalloc(&sys->Ms, (size_t)t.nnz));
    PG_TRY(dalloc(&sys->Kd, (size_t)n));
    PG_TRY(dalloc(&sys->Msd, (size_t)n));
    PG_TRY(dalloc(&sys->dflag, 4));
    auto up = [&](void* d, const void* h, size_t bytes) -> int {
        PG_HIP(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, s));
        return PETGEM_OK;
    };
    PG_TRY(up(sys->xyz, sys->xyz_h.data(), sys->xyz_h.size() * sizeof(double)));
    PG_TRY(up(sys->tets, sys->tets_h.data(), sys->tets_h.size() * sizeof(int32_t)));
    PG_TRY(up(sys->sigma, sigma, (size_t)T * sizeof(double)));
    PG_TRY(up(sys->row_ptr, t.row_ptr.data(), t.row_ptr.size() * sizeof(int32_t)));
    PG_TRY(up(sys->col, t.col.data(), t.col.size() * sizeof(int32_t)));
    PG_TRY(up(sys->diag_pos, t.diag_pos.data(), t.diag_pos.size() * sizeof(int32_t)));
    PG_TRY(up(sys->cptr, t.contrib_ptr.data(), t.contrib_ptr.size() * sizeof(int32_t)));
    PG_TRY(up(sys->cidx, t.contrib_idx.data(), t.contrib_idx.size() * sizeof(int32_t)));
    PG_TRY(up(sys->iptr, t.inc_ptr.data(), t.inc_ptr.size() * sizeof(int32_t)));
    PG_TRY(up(sys->islot, t.inc_slot.data(), t.inc_slot.size() * sizeof(int32_t)));
    int zero[4] = {0, 0, 0, 0};
    PG_TRY(up(sys->dflag, zero, sizeof(zero)));
    // the uploads read host vectors that die with `t`: wait for them
    PG_HIP(hipStreamSynchronize(s));
    return PETGEM_OK;
}

void release_system(petgem_system* sys) {
    if (!sys) return;
    dfree(sys->xyz); dfree(sys->tets); dfree(sys->sigma); dfree(sys->row_ptr); dfree(sys->col);
    dfree(sys->diag_pos); dfree(sys->cptr); dfree(sys->cidx); dfree(sys->iptr); dfree(sys->islot);
    dfree(sys->Kst); dfree(sys->Mst); dfree(sys->K); dfree(sys->Ms); dfree(sys->Kd); dfree(sys->Msd);
    sys->sell32.release();
    sys->ssor32.release();
    dfree(sys->K32); dfree(sys->Ms32); dfree(sys->Ahat); dfree(sys->dvec); dfree(sys->dinv);
    dfree(sys->Rst); dfree(sys->dflag); dfree(sys->tmp);
    dfree(sys->vox_tet); dfree(sys->vox_dof); dfree(sys->dof_mid); dfree(sys->dof_tan);
    sys->gw.release();
    release_block_work(sys->bw);
    sys->rxc.release();
}

// Locates the receivers on the host (cached while the same coordinates are
// passed again) and uploads their elements and DOFs.
int prepare_receivers(const petgem_solution* sol, const double* rx, int32_t n_rx) {
    petgem_system* sys = sol->sys;
    ReceiverCache& c = sys->rxc;
    if (c.n_rx != n_rx || std::memcmp(c.rx.data(), rx, sizeof(double) * 3 * (size_t)n_rx) != 0) {
        c.release();
        std::vector<int32_t> tet(n_rx);
        locate_points(sys->n_tets, sys->xyz_h.data(), sys->tets_h.data(), rx, n_rx, 1e-12, tet.data());
        std::vector<int32_t> dof(6 * (size_t)n_rx);
        for (int32_t r = 0; r < n_rx; ++r) {
            if (tet[r] < 0) {
                set_error("receiver " + std::to_string(r) + " lies outside the mesh");
                return PETGEM_RECEIVER_OUTSIDE;
            }
            for (int i = 0; i < 6; ++i) dof[6 * r + i] = sys->elem_dof_h[6 * (size_t)tet[r] + i];
        }
        PG_TRY(dalloc(&c.tet, (size_t)n_rx));
        PG_TRY(dalloc(&c.dof, 6 * (size_t)n_rx));
        PG_TRY(dalloc(&c.xyz, 3 * (size_t)n_rx));
        PG_HIP(hipMemcpy(c.tet, tet.data(), sizeof(int32_t) * n_rx, hipMemcpyHostToDevice));
        PG_HIP(hipMemcpy(c.dof, dof.data(), sizeof(int32_t) * 6 * n_rx, hipMemcpyHostToDevice));
        PG_HIP(hipMemcpy(c.xyz, rx, sizeof(double) * 3 * n_rx, hipMemcpyHostToDevice));
        c.rx.assign(rx, rx + 3 * (size_t)n_rx);
        c.n_rx = n_rx;
    }
    return PETGEM_OK;
}

}  // namespace

void set_error(const std::string& msg) { g_err = msg; }

}  // namespace petgem

using namespace petgem;

extern "C" {

const char* petgem_last_error(void) { return g_err.c_str(); }

void petgem_default_opts(petgem_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->method = PETGEM_GMRES;
    o->precision = PETGEM_FP64;
    o->restart = 30;
    o->max_iter = 20000;
    o->rtol = 1e-8;
    o->inner_rtol = 3e-5;
    o->use_graph = 1;
    o->profile = 0;
    o->verbose = 0;
    o->spmm_shape = 0;
    o->precond = PETGEM_JACOBI;
    o->omega = 1.0;
}

int petgem_assemble(const petgem_mesh* mesh, const double* sigma, double sigma_bg, void* stream,
                    petgem_system** out) {
    if (!out) { set_error("null output handle"); return PETGEM_INVALID_ARG; }
    *out = nullptr;
    if (!mesh || !mesh->xyz || !mesh->tets || !sigma || mesh->n_nodes <= 0 || mesh->n_tets <= 0) {
        set_error("mesh, coordinates, elements and conductivities are required");
        return PETGEM_INVALID_ARG;
    }
    if (!(sigma_bg > 0.0) || !std::isfinite(sigma_bg)) {
        set_error("background conductivity must be positive and finite");
        return PETGEM_INVALID_ARG;
    }
    for (int32_t t = 0; t < mesh->n_tets; ++t)
        if (!(sigma[t] > 0.0) || !std::isfinite(sigma[t])) {
            set_error("conductivity of element " + std::to_string(t) + " is not positive and finite");
            return PETGEM_INVALID_ARG;
        }
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = static_cast<hipStream_t>(stream);
    petgem_system* sys = new (std::nothrow) petgem_system();
    if (!sys) { set_error("host allocation failed"); return PETGEM_OUT_OF_MEMORY; }
    int rc = PETGEM_OK;
    {
        HostTopology topo;
        std::string err;
        rc = build_topology(mesh->n_nodes, mesh->n_tets, mesh->xyz, mesh->tets, topo, err);
        if (rc != PETGEM_OK) {
            set_error(err);
            delete sys;
            return rc;
        }
        (void)hipGetDevice(&sys->device);
        // the allocation-free entry point's scratch address on this device
        // (looked up once per device, with it current)
        char* scratch_base = nullptr;
        rc = noalloc_scratch(sys->device, &scratch_base);
        if (rc != PETGEM_OK) {
            delete sys;
            return rc;
        }
        sys->n_nodes = mesh->n_nodes;
        sys->n_tets = mesh->n_tets;
        sys->n_dof = topo.n_dof;
        sys->n_edges = topo.n_edges;
        sys->nnz = topo.nnz;
        sys->h_mean = topo.h_mean;
        sys->sigma_bg = sigma_bg;
        sys->xyz_h.assign(mesh->xyz, mesh->xyz + 3 * (size_t)mesh->n_nodes);
        sys->tets_h.assign(mesh->tets, mesh->tets + 4 * (size_t)mesh->n_tets);
        sys->elem_dof_h.resize(6 * (size_t)mesh->n_tets);
        for (size_t i = 0; i < sys->elem_dof_h.size(); ++i)
            sys->elem_dof_h[i] = topo.dof_of_edge[topo.elem_edge[i]];
        sys->dof_nodes_h.resize(2 * (size_t)topo.n_dof);
        for (int32_t r = 0; r < topo.n_dof; ++r) {
            sys->dof_nodes_h[2 * r] = topo.edge_lo[topo.edge_of_dof[r]];
            sys->dof_nodes_h[2 * r + 1] = topo.edge_hi[topo.edge_of_dof[r]];
        }
        sys->row_ptr_h = topo.row_ptr;
        rc = upload_topology(sys, topo, sigma, s);
    }
    sys->setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (rc == PETGEM_OK) rc = launch_assembly(sys, s);
    if (rc != PETGEM_OK) {
        release_system(sys);
        delete sys;
        return rc;
    }
    *out = sys;
    return PETGEM_OK;
}

int petgem_reassemble(petgem_system* sys, const double* sigma_dev, double sigma_bg, void* stream) {
    PG_TRY(check_sys(sys));
    if (!sigma_dev || !(sigma_bg > 0.0) || !std::isfinite(sigma_bg)) {
        set_error("reassemble needs device conductivities and a positive background");
        return PETGEM_INVALID_ARG;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    PG_HIP(hipMemcpyAsync(sys->sigma, sigma_dev, sizeof(double) * (size_t)sys->n_tets,
                          hipMemcpyDeviceToDevice, s));
    sys->sigma_bg = sigma_bg;
    return launch_assembly(sys, s);
}

int petgem_set_background(petgem_system* sys, const petgem_background* bg) {
    PG_TRY(check_sys(sys));
    if (!bg || (bg->layered != 0 && bg->layered != 1) ||
        (bg->layered && !(bg->sigma_above > 0.0 && bg->sigma_below > 0.0 && std::isfinite(bg->sigma_above) &&
                          std::isfinite(bg->sigma_below) && std::isfinite(bg->z0)))) {
        set_error("background: layered 0 or 1, positive finite conductivities, finite z0");
        return PETGEM_INVALID_ARG;
    }
    sys->layers.on = bg->layered;
    sys->layers.z0 = bg->z0;
    sys->layers.s_up = bg->sigma_above;
    sys->layers.s_dn = bg->sigma_below;
    return PETGEM_OK;
}

int petgem_rhs(petgem_system* sys, const petgem_source* src, int32_t n_src, void* b_dev, void* stream) {
    PG_TRY(check_sys(sys));
    if (!src || n_src <= 0 || !b_dev) { set_error("sources and output are required"); return PETGEM_INVALID_ARG; }
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int32_t k = 0; k < n_src; ++k) {
        PG_TRY(valid_source(src[k]));
        PG_TRY(launch_rhs(sys, src[k], static_cast<double2*>(b_dev) + (size_t)k * sys->n_dof, 1, s));
    }
    int flag = 0;
    PG_HIP(hipMemcpyAsync(&flag, sys->dflag, sizeof(int), hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    if (flag) {
        int zero = 0;
        PG_HIP(hipMemcpy(sys->dflag, &zero, sizeof(int), hipMemcpyHostToDevice));
        set_error("source within 1e-9 h of a quadrature point of an element with dsigma != 0");
        return PETGEM_SOURCE_SINGULAR;
    }
    return PETGEM_OK;
}

int petgem_rhs_noalloc(petgem_system* sys, const petgem_source* src, int32_t n_src, void* b_dev, void* stream) {
    PG_TRY(check_sys(sys));
    if (!src || n_src <= 0 || !b_dev) { set_error("sources and output are required"); return PETGEM_INVALID_ARG; }
    for (int32_t k = 0; k < n_src; ++k) PG_TRY(valid_source(src[k]));
    return rhs_noalloc(sys, src, n_src, static_cast<double2*>(b_dev), static_cast<hipStream_t>(stream));
}

int petgem_solve(petgem_system* sys, const petgem_source* src, int32_t n_src, const petgem_opts* opts,
                 const void* x0_dev, void* stream, petgem_solution** inout, petgem_stats* stats) {
    PG_TRY(check_sys(sys));
    if (!src || n_src <= 0 || !inout) { set_error("sources and a solution handle are required"); return PETGEM_INVALID_ARG; }
    petgem_opts o;
    if (opts) o = *opts; else petgem_default_opts(&o);
    if (o.method != PETGEM_GMRES && n_src > 256) {
        set_error("COCG solves at most 256 sources per call");
        return PETGEM_INVALID_ARG;
    }
    if (o.restart < 1 || o.restart > kMaxRestart || o.max_iter < 1 || !(o.rtol > 0.0) ||
        (o.method != PETGEM_GMRES && o.method != PETGEM_COCG && o.method != PETGEM_BCOCG &&
         o.method != PETGEM_SQMR) ||
        (o.precision != PETGEM_FP64 && o.precision != PETGEM_MIXED)) {
        set_error("invalid solver options");
        return PETGEM_INVALID_ARG;
    }
    if ((o.precond != PETGEM_JACOBI && o.precond != PETGEM_SSOR) ||
        (o.precond == PETGEM_SSOR && ((o.method != PETGEM_COCG && o.method != PETGEM_SQMR) ||
                                      !(o.omega > 0.0 && o.omega < 2.0))) ||
        (o.method == PETGEM_SQMR && o.precond != PETGEM_SSOR)) {
        set_error("precond: PETGEM_JACOBI, or PETGEM_SSOR with COCG or SQMR and 0 < omega < 2 (SQMR takes SSOR)");
        return PETGEM_INVALID_ARG;
    }
    for (int32_t k = 0; k < n_src; ++k) PG_TRY(valid_source(src[k]));
    hipStream_t s = static_cast<hipStream_t>(stream);
    petgem_solution* sol = *inout;
    if (sol && (sol->sys != sys || sol->n_src != n_src)) {
        set_error("solution handle belongs to another system or source count");
        return PETGEM_INVALID_ARG;
    }
    if (!sol) {
        sol = new (std::nothrow) petgem_solution();
        if (!sol) { set_error("host allocation failed"); return PETGEM_OUT_OF_MEMORY; }
        sol->sys = sys;
        sol->n_src = n_src;
        int rc = dalloc(&sol->x, (size_t)n_src * sys->n_dof);
        if (rc != PETGEM_OK) { delete sol; return rc; }
        *inout = sol;
    }
    sol->src.assign(src, src + n_src);
    sol->sigma_bg = sys->sigma_bg;
    sol->layers = sys->layers;
    if (stats) std::memset(stats, 0, sizeof(petgem_stats) * (size_t)n_src);
    const double2* x0 = static_cast<const double2*>(x0_dev);
    if (o.method == PETGEM_COCG || o.method == PETGEM_BCOCG || o.method == PETGEM_SQMR) {
        // A large block whose sources come in contiguous runs of one
        // frequency is solved one run at a time: the runs converge at very
        // different iteration counts (lower frequency, more iterations), and a
        // finished run then costs nothing (on the 6.9M-DOF, 96-source model:
        // 94 s instead of 112 s for one 96-column block).
        std::vector<int32_t> run = {0};
        for (int32_t k = 1; k < n_src; ++k)
            if (src[k].freq_hz != src[k - 1].freq_hz) run.push_back(k);
        run.push_back(n_src);
        bool contiguous = true;
        for (size_t a = 0; a + 1 < run.size(); ++a)
            for (size_t b = a + 1; b + 1 < run.size(); ++b)
                if (src[run[a]].freq_hz == src[run[b]].freq_hz) contiguous = false;
        // (block COCG solves one frequency per block, so always by runs)
        const bool split = run.size() > 2 && contiguous &&
                           ((int64_t)sys->n_dof * n_src >= kFreqRunMin || o.method == PETGEM_BCOCG);
        if (!split) return block_solve(sys, src, n_src, o, x0, sol->x, s, stats);
        int worst = PETGEM_OK;
        const size_t n = (size_t)sys->n_dof;
        for (size_t r = 0; r + 1 < run.size(); ++r) {
            const int32_t k0 = run[r], cnt = run[r + 1] - run[r];
            int rc = block_solve(sys, src + k0, cnt, o, x0 ? x0 + (size_t)k0 * n : nullptr, sol->x + (size_t)k0 * n,
                                 s, stats ? stats + k0 : nullptr);
            if (rc == PETGEM_NOT_CONVERGED || rc == PETGEM_NONFINITE) worst = rc;
            else if (rc != PETGEM_OK) return rc;
        }
        return worst;
    }
    int worst = PETGEM_OK;
    for (int32_t k = 0; k < n_src; ++k) {
        int rc = gmres_solve(sys, src[k], o, x0 ? x0 + (size_t)k * sys->n_dof : nullptr,
                             sol->x + (size_t)k * sys->n_dof, s, stats ? stats + k : nullptr);
        if (rc == PETGEM_NOT_CONVERGED || rc == PETGEM_NONFINITE) worst = rc;
        else if (rc != PETGEM_OK) return rc;
    }
    return worst;
}

int petgem_solve_many(petgem_system* const* systems, const petgem_source* src, int32_t n_sys,
                      const petgem_opts* opts, const void* const* x0_dev, void* stream, petgem_solution** sols,
                      petgem_stats* stats) {
    if (!systems || !src || n_sys <= 0 || !sols) { set_error("systems, sources and solutions are required"); return PETGEM_INVALID_ARG; }
    petgem_opts o;
    if (opts) o = *opts; else petgem_default_opts(&o);
    if (o.precond != PETGEM_JACOBI || o.method == PETGEM_SQMR) {
        set_error("the uneven batch takes COCG with the Jacobi preconditioner only");
        return PETGEM_INVALID_ARG;
    }
    for (int32_t k = 0; k < n_sys; ++k) {
        PG_TRY(check_sys(systems[k]));
        PG_TRY(valid_source(src[k]));
        petgem_solution*& sol = sols[k];
        if (sol && (sol->sys != systems[k] || sol->n_src != 1)) {
            set_error("solution handle belongs to another system or source count");
            return PETGEM_INVALID_ARG;
        }
        if (!sol) {
            sol = new (std::nothrow) petgem_solution();
            if (!sol) { set_error("host allocation failed"); return PETGEM_OUT_OF_MEMORY; }
            sol->sys = systems[k];
            sol->n_src = 1;
            PG_TRY(dalloc(&sol->x, (size_t)systems[k]->n_dof));
        }
        sol->src.assign(src + k, src + k + 1);
        sol->sigma_bg = systems[k]->sigma_bg;
        sol->layers = systems[k]->layers;
    }
    if (stats) std::memset(stats, 0, sizeof(petgem_stats) * (size_t)n_sys);
    return batch_solve(systems, src, n_sys, o, x0_dev, sols, static_cast<hipStream_t>(stream), stats);
}


int petgem_receivers(const petgem_solution* sol, const double* rx, int32_t n_rx, void* E_dev,
                     void* Es_dev, void* stream) {
    if (!sol || !sol->sys || !rx || n_rx <= 0 || !E_dev) {
        set_error("solution, receivers and output are required");
        return PETGEM_INVALID_ARG;
    }
    PG_TRY(prepare_receivers(sol, rx, n_rx));
    return launch_receivers(sol, n_rx, static_cast<double2*>(E_dev), static_cast<double2*>(Es_dev),
                            static_cast<hipStream_t>(stream));
}

int petgem_receivers_h(const petgem_solution* sol, const double* rx, int32_t n_rx, void* H_dev,
                       void* Hs_dev, void* stream) {
    if (!sol || !sol->sys || !rx || n_rx <= 0 || !H_dev) {
        set_error("solution, receivers and output are required");
        return PETGEM_INVALID_ARG;
    }
    PG_TRY(prepare_receivers(sol, rx, n_rx));
    return launch_receivers(sol, n_rx, static_cast<double2*>(H_dev), static_cast<double2*>(Hs_dev),
                            static_cast<hipStream_t>(stream), true);
}

int32_t petgem_num_dofs(const petgem_system* sys) { return sys ? sys->n_dof : -1; }
int64_t petgem_nnz(const petgem_system* sys) { return sys ? sys->nnz : -1; }
int32_t petgem_solution_nsrc(const petgem_solution* sol) { return sol ? sol->n_src : -1; }
const void* petgem_solution_x(const petgem_solution* sol) { return sol ? sol->x : nullptr; }
int petgem_solution_copy(const petgem_solution* sol, void* x_dev, void* stream) {
    if (!sol || !x_dev) { set_error("solution and output are required"); return PETGEM_INVALID_ARG; }
    PG_HIP(hipMemcpyAsync(x_dev, sol->x, sizeof(double2) * (size_t)sol->n_src * sol->sys->n_dof,
                          hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)));
    return PETGEM_OK;
}

int petgem_mesh_pattern(const petgem_mesh* mesh, int32_t* n_dof, int64_t* nnz, int32_t* dof_edges,
                        int32_t* row_ptr, int32_t* col) {
    if (!mesh || !n_dof || !nnz) { set_error("mesh and size outputs are required"); return PETGEM_INVALID_ARG; }
    HostTopology topo;
    std::string err;
    int rc = build_topology(mesh->n_nodes, mesh->n_tets, mesh->xyz, mesh->tets, topo, err);
    if (rc != PETGEM_OK) { set_error(err); return rc; }
    *n_dof = topo.n_dof;
    *nnz = topo.nnz;
    if (dof_edges)
        for (int32_t r = 0; r < topo.n_dof; ++r) {
            dof_edges[2 * r] = topo.edge_lo[topo.edge_of_dof[r]];
            dof_edges[2 * r + 1] = topo.edge_hi[topo.edge_of_dof[r]];
        }
    if (row_ptr) std::memcpy(row_ptr, topo.row_ptr.data(), sizeof(int32_t) * topo.row_ptr.size());
    if (col) std::memcpy(col, topo.col.data(), sizeof(int32_t) * topo.col.size());
    return PETGEM_OK;
}

int petgem_locate(const petgem_mesh* mesh, const double* pts, int32_t n_pts, double tol, int32_t* elem) {
    if (!mesh || !mesh->xyz || !mesh->tets || !pts || !elem || n_pts < 0) {
        set_error("mesh, points and output are required");
        return PETGEM_INVALID_ARG;
    }
    locate_points(mesh->n_tets, mesh->xyz, mesh->tets, pts, n_pts, tol, elem);
    return PETGEM_OK;
}

int petgem_tuning(const petgem_system* sys, int32_t* spmv_group, float* spmv_ms) {
    PG_TRY(check_sys(sys));
    if (spmv_group) *spmv_group = sys->spmv_tuned ? sys->spmv_group : 0;
    if (spmv_ms)
        for (int i = 0; i < 3; ++i) spmv_ms[i] = sys->spmv_tune_ms[i];
    return PETGEM_OK;
}

double petgem_setup_seconds(const petgem_system* sys) { return sys ? sys->setup_seconds : -1.0; }

int32_t petgem_ssor_colors(petgem_system* sys, int32_t* colors, void* stream) {
    PG_TRY(check_sys(sys));
    PG_TRY(ensure_ssor(sys, static_cast<hipStream_t>(stream)));
    PG_HIP(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    if (colors) std::memcpy(colors, sys->ssor32.color_h.data(), sizeof(int32_t) * (size_t)sys->n_dof);
    return sys->ssor32.nc;
}

int petgem_ssor_apply(petgem_system* sys, double freq, double omega, const void* r_dev, void* z_dev,
                      void* stream) {
    PG_TRY(check_sys(sys));
    if (!r_dev || !z_dev || r_dev == z_dev || !(freq > 0.0) || !(omega > 0.0 && omega < 2.0)) {
        set_error("petgem_ssor_apply: distinct vectors, freq > 0, 0 < omega < 2");
        return PETGEM_INVALID_ARG;
    }
    return ssor_apply1(sys, freq, omega, static_cast<const float2*>(r_dev), static_cast<float2*>(z_dev),
                       static_cast<hipStream_t>(stream));
}

int petgem_sync_probe(int32_t rounds, int32_t mode, int32_t* blocks, float* us_per_round, void* stream) {
    if (rounds < 1 || rounds > 100000 || (mode != 0 && mode != 1)) {
        set_error("petgem_sync_probe: 1 <= rounds <= 100000, mode 0 or 1");
        return PETGEM_INVALID_ARG;
    }
    return sync_probe(rounds, mode, blocks, us_per_round, static_cast<hipStream_t>(stream));
}

int32_t petgem_spmm_candidates(int32_t n_cols, int32_t sliced, int32_t* shapes, int32_t cap) {
    if (n_cols < 1 || cap < 0 || (cap > 0 && !shapes)) {
        set_error("petgem_spmm_candidates: n_cols >= 1 and a shapes array of cap entries");
        return PETGEM_INVALID_ARG;
    }
    return spmm_candidate_codes(n_cols, sliced != 0, shapes, cap);
}

int petgem_get_dof_edges(const petgem_system* sys, int32_t* edges) {
    PG_TRY(check_sys(sys));
    if (!edges) { set_error("null output"); return PETGEM_INVALID_ARG; }
    std::memcpy(edges, sys->dof_nodes_h.data(), sizeof(int32_t) * sys->dof_nodes_h.size());
    return PETGEM_OK;
}

int petgem_get_csr(const petgem_system* sys, int32_t* row_ptr, int32_t* col, double* K, double* Ms,
                   void* stream) {
    PG_TRY(check_sys(sys));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t nnz = (size_t)sys->nnz;
    if (row_ptr) PG_HIP(hipMemcpyAsync(row_ptr, sys->row_ptr, sizeof(int32_t) * (sys->n_dof + 1), hipMemcpyDeviceToHost, s));
    if (col) PG_HIP(hipMemcpyAsync(col, sys->col, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost, s));
    if (K) PG_HIP(hipMemcpyAsync(K, sys->K, sizeof(double) * nnz, hipMemcpyDeviceToHost, s));
    if (Ms) PG_HIP(hipMemcpyAsync(Ms, sys->Ms, sizeof(double) * nnz, hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    return PETGEM_OK;
}

int petgem_spmv(petgem_system* sys, double freq, const void* x_dev, void* y_dev, void* stream) {
    PG_TRY(check_sys(sys));
    if (!x_dev || !y_dev || !(freq > 0.0)) { set_error("spmv needs x, y and a positive frequency"); return PETGEM_INVALID_ARG; }
    hipStream_t s = static_cast<hipStream_t>(stream);
    PG_TRY(launch_freq_prep(sys, freq, s));
    PG_TRY(tune_spmv(sys, s));
    // A x = Ahat (D x) with the solver's CSR kernel
    PG_TRY(launch_spmv_unscaled(sys, static_cast<const double2*>(x_dev), static_cast<double2*>(y_dev), s));
    return PETGEM_OK;
}

void petgem_free_system(petgem_system* sys) {
    if (!sys) return;
    release_system(sys);
    delete sys;
}

void petgem_free_solution(petgem_solution* sol) {
    if (!sol) return;
    dfree(sol->x);
    delete sol;
}

}  // extern "C"
