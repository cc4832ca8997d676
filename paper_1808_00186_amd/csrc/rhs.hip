// Right-hand side (Section 3, eq. 9 with the primary field of Appendix A)
// and receiver interpolation (Section 3, eq. 8; Section 2, eq. 4).
//
// k_rhs_elem: one thread per tetrahedron; elements with sigma = sigma_bg
//   write zeros, the others evaluate the dipole field at the 4 points of the
//   degree-2 rule and integrate it against the 6 edge basis functions.
// k_rhs_gather: one thread per DOF sums its incident element entries in
//   increasing element order (deterministic, no atomics).
// k_receivers: one thread per receiver evaluates the 6 basis functions of its
//   element at the receiver and adds the primary field.
// k_receivers_h: the magnetic field H = curl E / (i w mu0) (Faraday's law of
//   Section 2 with e^{-iwt}): the curl of the secondary field is constant in
//   an element, sum_i e_i 2 s_i l_i grad lambda_a x grad lambda_b, and the
//   primary part is the dipole's analytic H.
#include "device.h"
#include "internal.h"

namespace petgem {

namespace {

constexpr int kE0[6] = {0, 0, 0, 1, 3, 2};
constexpr int kE1[6] = {1, 2, 3, 2, 1, 3};

struct SrcParams {
    double pos[3];
    double dir[3];
    double kappa;   // sqrt(w mu0 sigma_bg / 2)
    double pref;    // moment / (4 pi sigma_bg)
    double hpref;   // moment / (4 pi)
    double inv_wmu; // 1 / (w mu0)
};

SrcParams make_src(const petgem_source& s, double sigma_bg) {
    SrcParams p;
    for (int k = 0; k < 3; ++k) { p.pos[k] = s.pos[k]; p.dir[k] = s.dir[k]; }
    const double w = 2.0 * kPi * s.freq_hz;
    p.kappa = sqrt(w * kMu0 * sigma_bg * 0.5);
    p.pref = s.moment / (4.0 * kPi * sigma_bg);
    p.hpref = s.moment / (4.0 * kPi);
    p.inv_wmu = 1.0 / (w * kMu0);
    return p;
}

__global__ void __launch_bounds__(256)
k_rhs_elem(int T, const double* __restrict__ xyz, const int4* __restrict__ tets,
           const double* __restrict__ sigma, double sigma_bg, SrcParams sp, double wmu,
           double r_min, double2* __restrict__ Rst, int* __restrict__ flag) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    const double ds = sigma[t] - sigma_bg;
    if (ds == 0.0) {
#pragma unroll
        for (int i = 0; i < 6; ++i) Rst[(size_t)i * T + t] = make_double2(0.0, 0.0);
        return;
    }
    TetGeom G;
    tet_geometry(xyz, tets[t], G);
    // 4-point degree-2 rule: barycentric (a,b,b,b) and permutations, weights V/4
    const double qa = 0.58541019662496845446;   // (5 + 3 sqrt 5) / 20
    const double qb = 0.13819660112501051518;   // (5 - sqrt 5) / 20
    double2 R[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) R[i] = make_double2(0.0, 0.0);
    bool singular = false;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        double lam[4] = {qb, qb, qb, qb};
        lam[q] = qa;
        double x[3];
#pragma unroll
        for (int k = 0; k < 3; ++k)
            x[k] = lam[0] * G.X[0][k] + lam[1] * G.X[1][k] + lam[2] * G.X[2][k] + lam[3] * G.X[3][k];
        double d0 = x[0] - sp.pos[0], d1 = x[1] - sp.pos[1], d2 = x[2] - sp.pos[2];
        if (d0 * d0 + d1 * d1 + d2 * d2 <= r_min * r_min) singular = true;
        double2 E[3];
        dipole_E(x, sp.pos, sp.dir, sp.kappa, sp.pref, E);
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            const int a = kE0[i], b = kE1[i];
            double n0 = G.sl[i] * (lam[a] * G.g[b][0] - lam[b] * G.g[a][0]);
            double n1 = G.sl[i] * (lam[a] * G.g[b][1] - lam[b] * G.g[a][1]);
            double n2 = G.sl[i] * (lam[a] * G.g[b][2] - lam[b] * G.g[a][2]);
            R[i].x += n0 * E[0].x + n1 * E[1].x + n2 * E[2].x;
            R[i].y += n0 * E[0].y + n1 * E[1].y + n2 * E[2].y;
        }
    }
    if (singular) atomicOr(flag, 1);
    // i w mu0 dsigma (V/4) R  ->  multiply by i: (x, y) -> (-y, x)
    const double f = wmu * ds * G.vol * 0.25;
#pragma unroll
    for (int i = 0; i < 6; ++i) Rst[(size_t)i * T + t] = make_double2(-f * R[i].y, f * R[i].x);
}

__global__ void __launch_bounds__(256)
k_rhs_gather(int n, int T, const int32_t* __restrict__ iptr, const int32_t* __restrict__ islot,
             const double2* __restrict__ Rst, double2* __restrict__ b, int stride) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    double2 acc = make_double2(0.0, 0.0);
    const int32_t k1 = iptr[r + 1];
    // four incidences, then their entries, in flight at a time; the sum keeps
    // the list order
    for (int32_t k = iptr[r]; k < k1; k += 4) {
        int32_t sl[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) sl[q] = k + q < k1 ? islot[k + q] : -1;
        double2 v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int32_t t = sl[q] / 6, i = sl[q] - 6 * t;
            v[q] = sl[q] >= 0 ? Rst[(size_t)i * T + t] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (sl[q] >= 0) acc = cadd(acc, v[q]);
    }
    b[(size_t)r * stride] = acc;
}

__global__ void k_receivers(int n_rx, const double* __restrict__ rxyz, const int32_t* __restrict__ rtet,
                            const int32_t* __restrict__ rdof, const double* __restrict__ xyz,
                            const int4* __restrict__ tets, const double2* __restrict__ x,
                            SrcParams sp, double2* __restrict__ E, double2* __restrict__ Es) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rx) return;
    TetGeom G;
    tet_geometry(xyz, tets[rtet[r]], G);
    const double p[3] = {rxyz[3 * r], rxyz[3 * r + 1], rxyz[3 * r + 2]};
    double lam[4];
    lam[1] = lam[2] = lam[3] = 0.0;
#pragma unroll
    for (int v = 1; v < 4; ++v)
#pragma unroll
        for (int k = 0; k < 3; ++k) lam[v] += G.g[v][k] * (p[k] - G.X[0][k]);
    lam[0] = 1.0 - lam[1] - lam[2] - lam[3];
    double2 es[3] = {make_double2(0, 0), make_double2(0, 0), make_double2(0, 0)};
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        int d = rdof[6 * r + i];
        if (d < 0) continue;
        double2 v = x[d];
        const int a = kE0[i], b = kE1[i];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            double nk = G.sl[i] * (lam[a] * G.g[b][k] - lam[b] * G.g[a][k]);
            es[k].x += nk * v.x;
            es[k].y += nk * v.y;
        }
    }
    double2 ep[3];
    dipole_E(p, sp.pos, sp.dir, sp.kappa, sp.pref, ep);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        E[3 * r + k] = cadd(ep[k], es[k]);
        if (Es) Es[3 * r + k] = es[k];
    }
}

__global__ void k_receivers_h(int n_rx, const double* __restrict__ rxyz, const int32_t* __restrict__ rtet,
                              const int32_t* __restrict__ rdof, const double* __restrict__ xyz,
                              const int4* __restrict__ tets, const double2* __restrict__ x,
                              SrcParams sp, double2* __restrict__ H, double2* __restrict__ Hs) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rx) return;
    TetGeom G;
    tet_geometry(xyz, tets[rtet[r]], G);
    double2 cs[3] = {make_double2(0, 0), make_double2(0, 0), make_double2(0, 0)};
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        int d = rdof[6 * r + i];
        if (d < 0) continue;
        const double2 v = x[d];
        const int a = kE0[i], b = kE1[i];
        // curl N_i = 2 s_i l_i grad lambda_a x grad lambda_b
        const double c0 = 2.0 * G.sl[i] * (G.g[a][1] * G.g[b][2] - G.g[a][2] * G.g[b][1]);
        const double c1 = 2.0 * G.sl[i] * (G.g[a][2] * G.g[b][0] - G.g[a][0] * G.g[b][2]);
        const double c2 = 2.0 * G.sl[i] * (G.g[a][0] * G.g[b][1] - G.g[a][1] * G.g[b][0]);
        cs[0].x += c0 * v.x; cs[0].y += c0 * v.y;
        cs[1].x += c1 * v.x; cs[1].y += c1 * v.y;
        cs[2].x += c2 * v.x; cs[2].y += c2 * v.y;
    }
    const double p[3] = {rxyz[3 * r], rxyz[3 * r + 1], rxyz[3 * r + 2]};
    double2 hp[3];
    dipole_H(p, sp.pos, sp.dir, sp.kappa, sp.hpref, hp);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        // curl E_s / (i w mu0) = -i curl E_s / (w mu0): (x, y) -> (y, -x) / (w mu0)
        const double2 hs = make_double2(cs[k].y * sp.inv_wmu, -cs[k].x * sp.inv_wmu);
        H[3 * r + k] = cadd(hp[k], hs);
        if (Hs) Hs[3 * r + k] = hs;
    }
}

}  // namespace

// The element staging and the singular-source flag of one right-hand side,
// written where the caller says (the system's buffers, or the scratch of the
// allocation-free entry point).
int launch_rhs_into(petgem_system* sys, const petgem_source& src, double2* b, int b_stride, double2* Rst,
                    int* flag, hipStream_t s) {
    const int T = sys->n_tets;
    SrcParams sp = make_src(src, sys->sigma_bg);
    const double wmu = 2.0 * kPi * src.freq_hz * kMu0;
    if (sys->layers.on) {
        PG_TRY(launch_rhs_layered(sys, src, Rst, flag, s));
    } else {
        hipLaunchKernelGGL(k_rhs_elem, dim3(ceil_div(T, 256)), dim3(256), 0, s, T, sys->xyz,
                           reinterpret_cast<const int4*>(sys->tets), sys->sigma, sys->sigma_bg, sp, wmu,
                           1e-9 * sys->h_mean, Rst, flag);
        PG_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_rhs_gather, dim3(ceil_div(sys->n_dof, 256)), dim3(256), 0, s, sys->n_dof,
                       T, sys->iptr, sys->islot, Rst, b, b_stride);
    PG_HIP(hipGetLastError());
    return PETGEM_OK;
}

int launch_rhs(petgem_system* sys, const petgem_source& src, double2* b, int b_stride,
               hipStream_t s) {
    if (!sys->Rst) PG_TRY(dalloc(&sys->Rst, (size_t)6 * sys->n_tets));
    return launch_rhs_into(sys, src, b, b_stride, sys->Rst, sys->dflag, s);
}

int launch_receivers(const petgem_solution* sol, int32_t n_rx, double2* E, double2* Es,
                     hipStream_t s, bool magnetic) {
    const petgem_system* sys = sol->sys;
    if (sol->layers.on && magnetic) {
        set_error("the magnetic field over a layered background is not provided");
        return PETGEM_INVALID_ARG;
    }
    for (int32_t k = 0; k < sol->n_src; ++k) {
        SrcParams sp = make_src(sol->src[k], sol->sigma_bg);
        if (sol->layers.on) {
            PG_TRY(launch_receivers_layered(sol, k, n_rx, E + (size_t)k * n_rx * 3,
                                            Es ? Es + (size_t)k * n_rx * 3 : nullptr, s));
            continue;
        }
        if (magnetic) {
            hipLaunchKernelGGL(k_receivers_h, dim3(ceil_div(n_rx, 64)), dim3(64), 0, s, n_rx,
                               sys->rxc.xyz, sys->rxc.tet, sys->rxc.dof, sys->xyz,
                               reinterpret_cast<const int4*>(sys->tets),
                               sol->x + (size_t)k * sys->n_dof, sp, E + (size_t)k * n_rx * 3,
                               Es ? Es + (size_t)k * n_rx * 3 : nullptr);
            PG_HIP(hipGetLastError());
            continue;
        }
        hipLaunchKernelGGL(k_receivers, dim3(ceil_div(n_rx, 64)), dim3(64), 0, s, n_rx,
                           sys->rxc.xyz, sys->rxc.tet, sys->rxc.dof, sys->xyz,
                           reinterpret_cast<const int4*>(sys->tets),
                           sol->x + (size_t)k * sys->n_dof, sp, E + (size_t)k * n_rx * 3,
                           Es ? Es + (size_t)k * n_rx * 3 : nullptr);
        PG_HIP(hipGetLastError());
    }
    return PETGEM_OK;
}

}  // namespace petgem
