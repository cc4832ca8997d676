// Host mesh preprocessing (see mesh.h). Everything here is setup work done
// once per mesh; the per-conductivity and per-source work runs on the GPU.
#include "mesh.h"

#include <atomic>
#include <cmath>
#include <cstring>
#include <numeric>

#include "../../include/petgem.h"

namespace petgem {

namespace {

// Solve for the barycentric coordinates of p in tet (x0..x3): with
// J = [x1-x0, x2-x0, x3-x0] (columns), lambda_{1..3} = J^{-1} (p - x0) and
// lambda_0 = 1 - sum.
inline void barycentric(const double* x0, const double* x1, const double* x2,
                        const double* x3, const double* p, double lam[4]) {
    double a[3], b[3], c[3], d[3];
    for (int k = 0; k < 3; ++k) {
        a[k] = x1[k] - x0[k]; b[k] = x2[k] - x0[k]; c[k] = x3[k] - x0[k]; d[k] = p[k] - x0[k];
    }
    // J^{-1} rows are (b x c, c x a, a x b) / det with det = a . (b x c)
    double bc[3] = {b[1] * c[2] - b[2] * c[1], b[2] * c[0] - b[0] * c[2], b[0] * c[1] - b[1] * c[0]};
    double ca[3] = {c[1] * a[2] - c[2] * a[1], c[2] * a[0] - c[0] * a[2], c[0] * a[1] - c[1] * a[0]};
    double ab[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
    double det = a[0] * bc[0] + a[1] * bc[1] + a[2] * bc[2];
    lam[1] = (bc[0] * d[0] + bc[1] * d[1] + bc[2] * d[2]) / det;
    lam[2] = (ca[0] * d[0] + ca[1] * d[1] + ca[2] * d[2]) / det;
    lam[3] = (ab[0] * d[0] + ab[1] * d[1] + ab[2] * d[2]) / det;
    lam[0] = 1.0 - lam[1] - lam[2] - lam[3];
}

template <class T>
void exclusive_scan_inplace(std::vector<T>& v) {
    T run = 0;
    for (auto& x : v) { T c = x; x = run; run += c; }
}

}  // namespace

int build_topology(int32_t n_nodes, int32_t n_tets, const double* xyz,
                   const int32_t* tets, HostTopology& topo, std::string& err) {
    if (n_nodes <= 0 || n_tets <= 0 || !xyz || !tets) {
        err = "empty mesh";
        return PETGEM_INVALID_ARG;
    }
    if (int64_t(n_tets) * 21 >= (int64_t(1) << 31)) {
        err = "mesh too large for 32-bit gather indices (n_tets * 21 >= 2^31)";
        return PETGEM_INVALID_ARG;
    }
    const int64_t T = n_tets, N = n_nodes;
    for (int64_t i = 0; i < 4 * T; ++i) {
        if (tets[i] < 0 || tets[i] >= n_nodes) {
            err = "element " + std::to_string(i / 4) + " references node " +
                  std::to_string(tets[i]) + " outside [0, n_nodes)";
            return PETGEM_INVALID_ARG;
        }
    }
    topo = HostTopology();
    topo.n_nodes = n_nodes;
    topo.n_tets = n_tets;

    // ---- unique edges, bucketed by their lower node -------------------------
    std::vector<int32_t> bstart(N + 1, 0);
    for (int64_t t = 0; t < T; ++t)
        for (int i = 0; i < 6; ++i) {
            int32_t a = tets[4 * t + kLocalEdge[i][0]], b = tets[4 * t + kLocalEdge[i][1]];
            bstart[std::min(a, b) + 1]++;
        }
    for (int64_t i = 0; i < N; ++i) bstart[i + 1] += bstart[i];
    std::vector<int64_t> ent(6 * T);    // (hi << 32) | slot, sorted per bucket
    {
        std::vector<int32_t> cur(bstart.begin(), bstart.end() - 1);
        for (int64_t t = 0; t < T; ++t)
            for (int i = 0; i < 6; ++i) {
                int32_t a = tets[4 * t + kLocalEdge[i][0]], b = tets[4 * t + kLocalEdge[i][1]];
                int32_t lo = std::min(a, b), hi = std::max(a, b);
                if (lo == hi) {
                    err = "element " + std::to_string(t) + " repeats a node";
                    return PETGEM_DEGENERATE_ELEMENT;
                }
                ent[cur[lo]++] = (int64_t(hi) << 32) | int64_t(6 * t + i);
            }
    }
    std::vector<int32_t> ucount(N + 1, 0);
    parallel_for(N, [&](int64_t b, int64_t e) {
        for (int64_t lo = b; lo < e; ++lo) {
            std::sort(ent.begin() + bstart[lo], ent.begin() + bstart[lo + 1]);
            int32_t u = 0;
            for (int32_t k = bstart[lo]; k < bstart[lo + 1]; ++k)
                if (k == bstart[lo] || (ent[k] >> 32) != (ent[k - 1] >> 32)) ++u;
            ucount[lo + 1] = u;
        }
    });
    std::vector<int32_t>& ustart = ucount;   // becomes the prefix sum
    for (int64_t i = 0; i < N; ++i) ustart[i + 1] += ustart[i];
    const int32_t E = ustart[N];
    topo.n_edges = E;
    topo.edge_lo.resize(E);
    topo.edge_hi.resize(E);
    topo.elem_edge.assign(6 * T, -1);
    std::vector<int32_t> edge_inc_ptr(E + 1);
    parallel_for(N, [&](int64_t b, int64_t e) {
        for (int64_t lo = b; lo < e; ++lo) {
            int32_t id = ustart[lo] - 1;
            for (int32_t k = bstart[lo]; k < bstart[lo + 1]; ++k) {
                if (k == bstart[lo] || (ent[k] >> 32) != (ent[k - 1] >> 32)) {
                    ++id;
                    topo.edge_lo[id] = int32_t(lo);
                    topo.edge_hi[id] = int32_t(ent[k] >> 32);
                    edge_inc_ptr[id] = k;
                }
                topo.elem_edge[ent[k] & 0xffffffff] = id;
            }
        }
    });
    edge_inc_ptr[E] = int32_t(6 * T);
    auto find_edge = [&](int32_t a, int32_t b) -> int32_t {
        int32_t lo = std::min(a, b), hi = std::max(a, b);
        auto first = topo.edge_hi.begin() + ustart[lo], last = topo.edge_hi.begin() + ustart[lo + 1];
        auto it = std::lower_bound(first, last, hi);
        return (it != last && *it == hi) ? int32_t(it - topo.edge_hi.begin()) : -1;
    };

    // ---- geometry checks: non-degenerate elements --------------------------
    {
        double lsum = 0.0;
        for (int32_t e = 0; e < E; ++e) {
            const double* p = xyz + 3 * int64_t(topo.edge_lo[e]);
            const double* q = xyz + 3 * int64_t(topo.edge_hi[e]);
            lsum += std::sqrt((q[0] - p[0]) * (q[0] - p[0]) + (q[1] - p[1]) * (q[1] - p[1]) +
                              (q[2] - p[2]) * (q[2] - p[2]));
        }
        topo.h_mean = lsum / E;
        const double vmin = 1e-14 * topo.h_mean * topo.h_mean * topo.h_mean;
        std::atomic<int64_t> bad(-1);
        parallel_for(T, [&](int64_t b, int64_t e) {
            for (int64_t t = b; t < e; ++t) {
                const double* x0 = xyz + 3 * int64_t(tets[4 * t]);
                double a[3][3];
                for (int v = 1; v < 4; ++v)
                    for (int k = 0; k < 3; ++k) a[v - 1][k] = xyz[3 * int64_t(tets[4 * t + v]) + k] - x0[k];
                double det = a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) -
                             a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0]) +
                             a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]);
                if (!(std::fabs(det) / 6.0 > vmin)) {
                    int64_t exp = -1;
                    bad.compare_exchange_strong(exp, t);
                }
            }
        });
        if (bad.load() >= 0) {
            err = "degenerate element " + std::to_string(bad.load());
            return PETGEM_DEGENERATE_ELEMENT;
        }
    }

    // ---- boundary faces (faces of exactly one element) -> boundary edges ---
    std::vector<uint8_t> bnd(E, 0);
    {
        std::vector<int32_t> fstart(N + 1, 0);
        auto face_of = [&](int64_t t, int f, int32_t v[3]) {
            int k = 0;
            for (int j = 0; j < 4; ++j)
                if (j != f) v[k++] = tets[4 * t + j];
            std::sort(v, v + 3);
        };
        for (int64_t t = 0; t < T; ++t)
            for (int f = 0; f < 4; ++f) {
                int32_t v[3];
                face_of(t, f, v);
                fstart[v[0] + 1]++;
            }
        for (int64_t i = 0; i < N; ++i) fstart[i + 1] += fstart[i];
        std::vector<int64_t> fent(4 * T);
        std::vector<int32_t> cur(fstart.begin(), fstart.end() - 1);
        for (int64_t t = 0; t < T; ++t)
            for (int f = 0; f < 4; ++f) {
                int32_t v[3];
                face_of(t, f, v);
                fent[cur[v[0]]++] = int64_t(v[1]) * N + v[2];
            }
        std::atomic<int> topo_err(0);
        std::vector<std::vector<int32_t>> marks(16);
        std::atomic<int> next_tid(0);
        parallel_for(N, [&](int64_t b, int64_t e) {
            std::vector<int32_t> mine;
            for (int64_t p = b; p < e; ++p) {
                auto first = fent.begin() + fstart[p], last = fent.begin() + fstart[p + 1];
                std::sort(first, last);
                for (auto it = first; it != last;) {
                    auto jt = it;
                    while (jt != last && *jt == *it) ++jt;
                    int64_t cnt = jt - it;
                    if (cnt > 2) topo_err = 1;
                    if (cnt == 1) {
                        int32_t q = int32_t(*it / N), r = int32_t(*it % N);
                        mine.push_back(find_edge(int32_t(p), q));
                        mine.push_back(find_edge(int32_t(p), r));
                        mine.push_back(find_edge(q, r));
                    }
                    it = jt;
                }
            }
            marks[next_tid++] = std::move(mine);
        });
        if (topo_err) {
            err = "a face is shared by more than two elements";
            return PETGEM_MESH_TOPOLOGY;
        }
        for (auto& m : marks)
            for (int32_t e : m) bnd[e] = 1;
    }

    // ---- interior DOF numbering along a Morton (Z-order) curve of the edge
    //      midpoints: consecutive rows are spatially compact, so a tile of rows
    //      gathers a small neighbourhood of x and shares it in cache ----------
    {
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (int64_t v = 0; v < N; ++v)
            for (int k = 0; k < 3; ++k) {
                lo[k] = std::min(lo[k], xyz[3 * v + k]);
                hi[k] = std::max(hi[k], xyz[3 * v + k]);
            }
        std::vector<std::pair<uint64_t, int32_t>> key;
        key.reserve(E);
        for (int32_t e = 0; e < E; ++e) {
            if (bnd[e]) continue;
            uint64_t code = 0;
            uint32_t q[3];
            for (int k = 0; k < 3; ++k) {
                const double m = 0.5 * (xyz[3 * int64_t(topo.edge_lo[e]) + k] + xyz[3 * int64_t(topo.edge_hi[e]) + k]);
                const double t = hi[k] > lo[k] ? (m - lo[k]) / (hi[k] - lo[k]) : 0.0;
                q[k] = uint32_t(std::min(std::max(t, 0.0), 1.0) * double((1u << 21) - 1));
            }
            for (int b = 20; b >= 0; --b)
                for (int k = 0; k < 3; ++k) code = (code << 1) | ((q[k] >> b) & 1u);
            key.emplace_back(code, e);
        }
        std::sort(key.begin(), key.end());
        topo.dof_of_edge.assign(E, -1);
        topo.edge_of_dof.resize(key.size());
        for (size_t r = 0; r < key.size(); ++r) {
            topo.edge_of_dof[r] = key[r].second;
            topo.dof_of_edge[key[r].second] = int32_t(r);
        }
    }
    const int32_t n = int32_t(topo.edge_of_dof.size());
    topo.n_dof = n;
    if (n == 0) {
        err = "mesh has no interior edge";
        return PETGEM_INVALID_ARG;
    }

    // ---- DOF -> incident (element, local edge) slots, increasing element ----
    topo.inc_ptr.assign(n + 1, 0);
    for (int32_t r = 0; r < n; ++r) {
        int32_t e = topo.edge_of_dof[r];
        topo.inc_ptr[r + 1] = topo.inc_ptr[r] + (edge_inc_ptr[e + 1] - edge_inc_ptr[e]);
    }
    topo.inc_slot.resize(topo.inc_ptr[n]);
    parallel_for(n, [&](int64_t b, int64_t e) {
        for (int64_t r = b; r < e; ++r) {
            int32_t ed = topo.edge_of_dof[r];
            int32_t o = topo.inc_ptr[r];
            for (int32_t k = edge_inc_ptr[ed]; k < edge_inc_ptr[ed + 1]; ++k)
                topo.inc_slot[o++] = int32_t(ent[k] & 0xffffffff);
        }
    });
    std::vector<int64_t>().swap(ent);

    // ---- CSR pattern: columns of row r are the interior edges sharing an
    //      element with edge r ---------------------------------------------
    auto row_columns = [&](int32_t r, std::vector<int32_t>& cols) {
        cols.clear();
        for (int32_t k = topo.inc_ptr[r]; k < topo.inc_ptr[r + 1]; ++k) {
            int32_t t = topo.inc_slot[k] / 6;
            for (int j = 0; j < 6; ++j) {
                int32_t d = topo.dof_of_edge[topo.elem_edge[6 * int64_t(t) + j]];
                if (d >= 0) cols.push_back(d);
            }
        }
        std::sort(cols.begin(), cols.end());
        cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
    };
    topo.row_ptr.assign(n + 1, 0);
    parallel_for(n, [&](int64_t b, int64_t e) {
        std::vector<int32_t> cols;
        for (int64_t r = b; r < e; ++r) {
            row_columns(int32_t(r), cols);
            topo.row_ptr[r + 1] = int32_t(cols.size());
        }
    });
    {
        int64_t run = 0;
        for (int32_t r = 0; r <= n; ++r) {
            int64_t c = topo.row_ptr[r];
            run += c;
            if (run >= (int64_t(1) << 31)) {
                err = "too many nonzeros for 32-bit CSR offsets";
                return PETGEM_INVALID_ARG;
            }
            topo.row_ptr[r] = int32_t(run);
        }
    }
    topo.nnz = topo.row_ptr[n];
    topo.col.resize(topo.nnz);
    topo.diag_pos.resize(n);
    std::vector<int32_t> ccount(topo.nnz + 1, 0);
    parallel_for(n, [&](int64_t b, int64_t e) {
        std::vector<int32_t> cols;
        for (int64_t r = b; r < e; ++r) {
            row_columns(int32_t(r), cols);
            std::copy(cols.begin(), cols.end(), topo.col.begin() + topo.row_ptr[r]);
            topo.diag_pos[r] = topo.row_ptr[r] +
                int32_t(std::lower_bound(cols.begin(), cols.end(), int32_t(r)) - cols.begin());
            // contributions per nonzero: one per shared element
            for (int32_t k = topo.inc_ptr[r]; k < topo.inc_ptr[r + 1]; ++k) {
                int32_t t = topo.inc_slot[k] / 6;
                for (int j = 0; j < 6; ++j) {
                    int32_t d = topo.dof_of_edge[topo.elem_edge[6 * int64_t(t) + j]];
                    if (d < 0) continue;
                    int32_t pos = topo.row_ptr[r] +
                        int32_t(std::lower_bound(cols.begin(), cols.end(), d) - cols.begin());
                    ccount[pos + 1]++;
                }
            }
        }
    });
    for (int64_t i = 0; i < topo.nnz; ++i) {
        ccount[i + 1] += ccount[i];
        if (ccount[i + 1] < 0) {
            err = "too many element contributions for 32-bit offsets";
            return PETGEM_INVALID_ARG;
        }
    }
    topo.contrib_ptr = ccount;
    topo.contrib_idx.resize(ccount[topo.nnz]);
    parallel_for(n, [&](int64_t b, int64_t e) {
        std::vector<int32_t> curpos;
        for (int64_t r = b; r < e; ++r) {
            int32_t r0 = topo.row_ptr[r], r1 = topo.row_ptr[r + 1];
            curpos.assign(topo.contrib_ptr.begin() + r0, topo.contrib_ptr.begin() + r1);
            for (int32_t k = topo.inc_ptr[r]; k < topo.inc_ptr[r + 1]; ++k) {
                int32_t slot = topo.inc_slot[k];
                int32_t t = slot / 6, i = slot % 6;
                for (int j = 0; j < 6; ++j) {
                    int32_t d = topo.dof_of_edge[topo.elem_edge[6 * int64_t(t) + j]];
                    if (d < 0) continue;
                    int32_t pos = int32_t(std::lower_bound(topo.col.begin() + r0, topo.col.begin() + r1, d) -
                                          topo.col.begin());
                    topo.contrib_idx[curpos[pos - r0]++] = packed_index(i, j) * n_tets + t;
                }
            }
        }
    });
    return PETGEM_OK;
}

void locate_points(int32_t n_tets, const double* xyz, const int32_t* tets,
                   const double* pts, int32_t n_pts, double tol, int32_t* elem) {
    for (int32_t r = 0; r < n_pts; ++r) elem[r] = -1;
    // Parallel over element chunks; the lowest hit per point wins.
    std::vector<std::atomic<int64_t>> best(n_pts);
    for (auto& b : best) b = INT64_MAX;
    parallel_for(n_tets, [&](int64_t b, int64_t e) {
        for (int64_t t = b; t < e; ++t) {
            const double* X[4];
            double lo[3], hi[3];
            for (int v = 0; v < 4; ++v) X[v] = xyz + 3 * int64_t(tets[4 * t + v]);
            for (int k = 0; k < 3; ++k) {
                lo[k] = std::min(std::min(X[0][k], X[1][k]), std::min(X[2][k], X[3][k]));
                hi[k] = std::max(std::max(X[0][k], X[1][k]), std::max(X[2][k], X[3][k]));
            }
            for (int32_t r = 0; r < n_pts; ++r) {
                const double* p = pts + 3 * r;
                bool in = true;
                for (int k = 0; k < 3; ++k) {
                    double pad = 1e-9 * (hi[k] - lo[k] + 1.0);
                    if (p[k] < lo[k] - pad || p[k] > hi[k] + pad) in = false;
                }
                if (!in) continue;
                double lam[4];
                barycentric(X[0], X[1], X[2], X[3], p, lam);
                if (lam[0] >= -tol && lam[1] >= -tol && lam[2] >= -tol && lam[3] >= -tol) {
                    int64_t cur = best[r].load();
                    while (t < cur && !best[r].compare_exchange_weak(cur, t)) {}
                }
            }
        }
    });
    for (int32_t r = 0; r < n_pts; ++r)
        if (best[r].load() != INT64_MAX) elem[r] = int32_t(best[r].load());
}

}  // namespace petgem
