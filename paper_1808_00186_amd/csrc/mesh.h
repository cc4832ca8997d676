// Host-side mesh preprocessing of the edge-FEM path: unique edges with their
// global orientation (Appendix B, eq. B.15), boundary faces and Dirichlet
// edges (Section 2), interior DOF numbering, the CSR sparsity pattern of the
// global system (the "sparsity structure" of the parameters file, Section 4)
// and the deterministic gather lists that let the GPU assemble without
// atomics. Plain C++17, no GPU calls.
#pragma once
#include <algorithm>
#include <cstdint>
#include <thread>
#include <string>
#include <vector>

namespace petgem {

// Local edges of the tetrahedron (Appendix B, eqs. B.1-B.6), vertices 0..3:
// e1 (0,1), e2 (0,2), e3 (0,3), e4 (1,2), e5 (3,1), e6 (2,3).
constexpr int kLocalEdge[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {3, 1}, {2, 3}};

// Index of the (i, j), i <= j, entry of a symmetric 6x6 element matrix in its
// packed upper triangle (21 entries).
inline int packed_index(int i, int j) {
    if (i > j) { int t = i; i = j; j = t; }
    return i * 6 - (i * (i - 1)) / 2 + (j - i);
}

struct HostTopology {
    int32_t n_nodes = 0, n_tets = 0, n_edges = 0, n_dof = 0;
    int64_t nnz = 0;
    double h_mean = 0.0;                 // mean edge length (for scale-aware checks)
    std::vector<int32_t> edge_lo, edge_hi;   // [n_edges], lo < hi
    std::vector<int32_t> elem_edge;          // [T][6]
    std::vector<int32_t> dof_of_edge;        // [n_edges], -1 on the boundary
    std::vector<int32_t> edge_of_dof;        // [n_dof]
    // CSR of the interior-edge system
    std::vector<int32_t> row_ptr;            // [n_dof + 1]
    std::vector<int32_t> col;                // [nnz]
    std::vector<int32_t> diag_pos;           // [n_dof]
    // nnz -> element-matrix entries: staging index k * T + t (k = packed
    // index of the local pair), in increasing element order
    std::vector<int32_t> contrib_ptr;        // [nnz + 1]
    std::vector<int32_t> contrib_idx;
    // DOF -> incident (element, local edge) slots t * 6 + i, increasing t
    std::vector<int32_t> inc_ptr;            // [n_dof + 1]
    std::vector<int32_t> inc_slot;
};

// Returns 0 or a PETGEM_* error code with a message in `err`.
int build_topology(int32_t n_nodes, int32_t n_tets, const double* xyz,
                   const int32_t* tets, HostTopology& topo, std::string& err);

// Point location: for each point, the lowest element id whose barycentric
// coordinates are all >= -tol, or -1 (the GPU recomputes the coordinates
// from the vertices).
void locate_points(int32_t n_tets, const double* xyz, const int32_t* tets,
                   const double* pts, int32_t n_pts, double tol, int32_t* elem);

// Runs fn(begin, end) over [0, n) in contiguous chunks on the hardware
// threads (at most 16).
template <class F>
void parallel_for(int64_t n, F&& fn) {
    unsigned hw = std::thread::hardware_concurrency();
    int64_t nt = hw == 0 ? 1 : (hw > 16 ? 16 : hw);
    if (n < 4096 || nt == 1) { fn(int64_t(0), n); return; }
    std::vector<std::thread> th;
    int64_t chunk = (n + nt - 1) / nt;
    for (int64_t t = 0; t < nt; ++t) {
        int64_t b = t * chunk, e = std::min(n, b + chunk);
        if (b >= e) break;
        th.emplace_back([&fn, b, e]() { fn(b, e); });
    }
    for (auto& x : th) x.join();
}

}  // namespace petgem
