// Right-hand side and receiver fields over a layered background of two
// half-spaces (the layered primary field; see the comment below). The
// whole-space case is in rhs.hip.
#include <cmath>

#include "device.h"
#include "internal.h"

namespace petgem {

namespace {

constexpr int kLE0[6] = {0, 0, 0, 1, 3, 2};
constexpr int kLE1[6] = {1, 2, 3, 2, 1, 3};

struct LSrc {
    double pos[3];
    double dir[3];
    double w;      // angular frequency
    double mom;    // moment I dS
};

// ------------------------------------------------- layered background
// Primary field of the dipole over two half-spaces (sigma_1 above z0, holding
// the source; sigma_2 below), from the TE / TM split of the whole-space field
// at the flat interface (Section 2: the primary field is that of the
// background model). With kappa the horizontal wavenumber,
// u_j = sqrt(kappa^2 - i w mu0 sigma_j) (Re u_j > 0),
//   r_TE = (u1 - u2)/(u1 + u2),   r_TM = (s2 u1 - s1 u2)/(s2 u1 + s1 u2),
//   t_TE = 2 u1/(u1 + u2),        t_TM = 2 s1 u1/(s2 u1 + s1 u2),
// and Hankel transforms in the horizontal offset rho at angle phi, c = m/(8 pi s1):
// above: E = E_whole-space(s1) + E_r with Z = (z - z0) + (zs - z0),
//   A_n = int k1^2 r_TE/u1 e^{-u1 Z} J_n k dk,  B_n = int u1 r_TM e^{-u1 Z} J_n k dk,
//   E1 = int r_TM e^{-u1 Z} J_1 k^2 dk,        V0 = int r_TM k^3/u1 e^{-u1 Z} J_0 dk;
//   x dipole: (c (A0 + B0 + cos2phi (A2 - B2)), c sin2phi (A2 - B2), -2c cos phi E1),
//   y dipole: (c sin2phi (A2 - B2), c (A0 + B0 - cos2phi (A2 - B2)), -2c sin phi E1),
//   z dipole: (2c cos phi E1, 2c sin phi E1, 2c V0);
// below, with e = exp(u2 (z - z0) - u1 (zs - z0)): the same with t for r,
//   TA_n = int k1^2 t_TE/u1 e J_n k dk, TB_n = int u2 t_TM e J_n k dk,
//   TE1 = int t_TM e J_1 k^2 dk, VE1 = int t_TM u2/u1 e J_1 k^2 dk, VV0 = int t_TM k^3/u1 e J_0 dk;
//   x dipole: (c (TA0 - TB0 + cos2phi (TA2 + TB2)), c sin2phi (TA2 + TB2), -2c cos phi TE1),
//   y dipole: (c sin2phi (TA2 + TB2), c (TA0 - TB0 - cos2phi (TA2 + TB2)), -2c sin phi TE1),
//   z dipole: (-2c cos phi VE1, -2c sin phi VE1, 2c VV0).
// Quadrature: 16-point Gauss-Legendre panels over [0, kmax], kmax = 50 /
// (decay length) (the exponential below e^-50 there), panels of width
// min(0.2 min|k_j|, pi / (2.5 rho)) up to 10 max|k_j| and min(pi / (2.5 rho),
// (kmax - that) / 48) beyond; the 64 lanes of a wavefront share the nodes
// and the sums are reduced by shuffles in a fixed order.
struct GL16 {
    double x[16], w[16];   // nodes and weights on [-1, 1]
};

__device__ __forceinline__ double2 csqrt_p(double2 z) {   // principal branch
    const double r = hypot(z.x, z.y);
    const double t = sqrt(0.5 * (r + fabs(z.x)));
    if (t == 0.0) return make_double2(0.0, 0.0);
    if (z.x >= 0.0) return make_double2(t, z.y / (2.0 * t));
    return make_double2(fabs(z.y) / (2.0 * t), copysign(t, z.y));
}

__device__ __forceinline__ double2 cexp_(double2 z) {
    double s, c;
    sincos(z.y, &s, &c);
    const double e = exp(z.x);
    return make_double2(e * c, e * s);
}

// E_p at x; called by all 64 lanes of a wavefront with the same x, every
// lane gets the result.
__device__ void layered_E(const double x[3], const LSrc& sp, const Layers L, const GL16& gl, double2 E[3]) {
    const int lane = threadIdx.x & 63;
    const double w = sp.w;
    const double dx = x[0] - sp.pos[0], dy = x[1] - sp.pos[1];
    const double rho = sqrt(dx * dx + dy * dy);
    const double cph = rho > 0.0 ? dx / rho : 1.0, sph = rho > 0.0 ? dy / rho : 0.0;
    const double c2 = cph * cph - sph * sph, s2 = 2.0 * sph * cph;
    const double z = x[2] - L.z0, zs = sp.pos[2] - L.z0;
    const bool upper = z >= 0.0;
    const double dec = upper ? z + zs : zs - z;
    const double kmax = 50.0 / dec;
    const double s1 = L.s_up, s2s = L.s_dn;
    const double2 k1s = make_double2(0.0, w * kMu0 * s1), k2s = make_double2(0.0, w * kMu0 * s2s);
    const double ka1 = sqrt(w * kMu0 * s1), ka2 = sqrt(w * kMu0 * s2s);
    const double per = rho > 0.0 ? kPi / (2.5 * rho) : 1e300;
    const double kA = fmin(10.0 * fmax(ka1, ka2), kmax);
    const int nA = (int)ceil(kA / fmin(0.2 * fmin(ka1, ka2), per));
    const double hA = kA / nA;
    const int nB = kmax > kA ? (int)ceil((kmax - kA) / fmin(per, (kmax - kA) / 48.0)) : 0;
    const double hB = nB > 0 ? (kmax - kA) / nB : 0.0;
    const int N = 16 * (nA + nB);
    double2 I[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) I[j] = make_double2(0.0, 0.0);
    for (int n = lane; n < N; n += 64) {
        const int pnl = n >> 4, q = n & 15;
        const double a = pnl < nA ? pnl * hA : kA + (pnl - nA) * hB;
        const double h = pnl < nA ? hA : hB;
        const double kap = a + 0.5 * h * (1.0 + gl.x[q]);
        const double wt = 0.5 * h * gl.w[q];
        const double k2 = kap * kap;
        const double2 u1 = csqrt_p(make_double2(k2 - k1s.x, -k1s.y));
        const double2 u2 = csqrt_p(make_double2(k2 - k2s.x, -k2s.y));
        const double xr = kap * rho;
        const double j0v = j0(xr), j1v = j1(xr);
        const double j2v = xr > 1e-6 ? 2.0 * j1v / xr - j0v : 0.125 * xr * xr;
        const double2 iu1 = cdiv(make_double2(1.0, 0.0), u1);
        const double2 den = cadd(cscale(u1, s2s), cscale(u2, s1));
        if (upper) {
            const double2 rte = cdiv(csub(u1, u2), cadd(u1, u2));
            const double2 rtm = cdiv(csub(cscale(u1, s2s), cscale(u2, s1)), den);
            const double2 ex = cexp_(cscale(u1, -(z + zs)));
            const double2 fa = cscale(cmul(cmul(k1s, cmul(rte, iu1)), ex), kap * wt);
            const double2 fb = cscale(cmul(cmul(u1, rtm), ex), kap * wt);
            I[0] = cadd(I[0], cscale(fa, j0v));
            I[1] = cadd(I[1], cscale(fa, j2v));
            I[2] = cadd(I[2], cscale(fb, j0v));
            I[3] = cadd(I[3], cscale(fb, j2v));
            I[4] = cadd(I[4], cscale(cmul(rtm, ex), j1v * k2 * wt));
            I[5] = cadd(I[5], cscale(cmul(cmul(rtm, iu1), ex), k2 * kap * j0v * wt));
        } else {
            const double2 tte = cdiv(cscale(u1, 2.0), cadd(u1, u2));
            const double2 ttm = cdiv(cscale(u1, 2.0 * s1), den);
            const double2 ex = cexp_(csub(cscale(u2, z), cscale(u1, zs)));
            const double2 fa = cscale(cmul(cmul(k1s, cmul(tte, iu1)), ex), kap * wt);
            const double2 fb = cscale(cmul(cmul(u2, ttm), ex), kap * wt);
            I[0] = cadd(I[0], cscale(fa, j0v));
            I[1] = cadd(I[1], cscale(fa, j2v));
            I[2] = cadd(I[2], cscale(fb, j0v));
            I[3] = cadd(I[3], cscale(fb, j2v));
            const double2 te = cmul(ttm, ex);
            I[4] = cadd(I[4], cscale(te, j1v * k2 * wt));
            I[5] = cadd(I[5], cscale(cmul(cmul(te, u2), iu1), j1v * k2 * wt));
            I[6] = cadd(I[6], cscale(cmul(te, iu1), k2 * kap * j0v * wt));
        }
    }
#pragma unroll
    for (int j = 0; j < 7; ++j) { I[j].x = wave_sum(I[j].x); I[j].y = wave_sum(I[j].y); }
    const double c = sp.mom / (8.0 * kPi * s1);
    const double* p = sp.dir;
    double2 hx[3], hy[3], vz[3];
    if (upper) {
        const double2 S0 = cadd(I[0], I[2]), D2 = csub(I[1], I[3]);
        hx[0] = cscale(cadd(S0, cscale(D2, c2)), c); hx[1] = cscale(D2, c * s2); hx[2] = cscale(I[4], -2.0 * c * cph);
        hy[0] = cscale(D2, c * s2); hy[1] = cscale(csub(S0, cscale(D2, c2)), c); hy[2] = cscale(I[4], -2.0 * c * sph);
        vz[0] = cscale(I[4], 2.0 * c * cph); vz[1] = cscale(I[4], 2.0 * c * sph); vz[2] = cscale(I[5], 2.0 * c);
        double2 Ew[3];
        dipole_E(x, sp.pos, sp.dir, sqrt(0.5 * w * kMu0 * s1), sp.mom / (4.0 * kPi * s1), Ew);
#pragma unroll
        for (int k = 0; k < 3; ++k)
            E[k] = cadd(Ew[k], cadd(cadd(cscale(hx[k], p[0]), cscale(hy[k], p[1])), cscale(vz[k], p[2])));
    } else {
        const double2 S0 = csub(I[0], I[2]), D2 = cadd(I[1], I[3]);
        hx[0] = cscale(cadd(S0, cscale(D2, c2)), c); hx[1] = cscale(D2, c * s2); hx[2] = cscale(I[4], -2.0 * c * cph);
        hy[0] = cscale(D2, c * s2); hy[1] = cscale(csub(S0, cscale(D2, c2)), c); hy[2] = cscale(I[4], -2.0 * c * sph);
        vz[0] = cscale(I[5], -2.0 * c * cph); vz[1] = cscale(I[5], -2.0 * c * sph); vz[2] = cscale(I[6], 2.0 * c);
#pragma unroll
        for (int k = 0; k < 3; ++k)
            E[k] = cadd(cadd(cscale(hx[k], p[0]), cscale(hy[k], p[1])), cscale(vz[k], p[2]));
    }
}

// Right-hand side, one wavefront per element: dsigma_q = sigma_e -
// sigma_b(z_q) at each point of the 4-point rule (weights V/4), the layered
// E_p where it is non-zero; entries i w mu0 (V/4) sum_q dsigma_q N_i . E_p
// into Rst[i][t] (element-major planes, as the whole-space kernel).
__global__ void __launch_bounds__(64)
k_rhs_layered(int T, const double* __restrict__ xyz, const int4* __restrict__ tets, const double* __restrict__ sigma,
              Layers L, LSrc sp, GL16 gl, double r_min, double2* __restrict__ Rst, int* __restrict__ flag) {
    const int t = blockIdx.x;
    TetGeom G;
    tet_geometry(xyz, tets[t], G);
    const double qa = 0.58541019662496845446, qb = 0.13819660112501051518;   // (5 +- 3 sqrt 5)/20, (5 - sqrt 5)/20
    double ds[4];
    bool any = false;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        double zq = 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) zq += (v == q ? qa : qb) * G.X[v][2];
        ds[q] = sigma[t] - (zq >= L.z0 ? L.s_up : L.s_dn);
        any = any || ds[q] != 0.0;
    }
    double2 R[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) R[i] = make_double2(0.0, 0.0);
    bool singular = false;
    if (any) {
        for (int q = 0; q < 4; ++q) {
            if (ds[q] == 0.0) continue;   // the same in every lane
            double lam[4] = {qb, qb, qb, qb};
            lam[q] = qa;
            double x[3];
#pragma unroll
            for (int k = 0; k < 3; ++k)
                x[k] = lam[0] * G.X[0][k] + lam[1] * G.X[1][k] + lam[2] * G.X[2][k] + lam[3] * G.X[3][k];
            const double d0 = x[0] - sp.pos[0], d1 = x[1] - sp.pos[1], d2 = x[2] - sp.pos[2];
            if (d0 * d0 + d1 * d1 + d2 * d2 <= r_min * r_min) singular = true;
            double2 E[3];
            layered_E(x, sp, L, gl, E);
#pragma unroll
            for (int i = 0; i < 6; ++i) {
                const int a = kLE0[i], b = kLE1[i];
                const double n0 = G.sl[i] * (lam[a] * G.g[b][0] - lam[b] * G.g[a][0]);
                const double n1 = G.sl[i] * (lam[a] * G.g[b][1] - lam[b] * G.g[a][1]);
                const double n2 = G.sl[i] * (lam[a] * G.g[b][2] - lam[b] * G.g[a][2]);
                R[i].x += ds[q] * (n0 * E[0].x + n1 * E[1].x + n2 * E[2].x);
                R[i].y += ds[q] * (n0 * E[0].y + n1 * E[1].y + n2 * E[2].y);
            }
        }
    }
    if (threadIdx.x != 0) return;
    if (singular) atomicOr(flag, 1);
    // i w mu0 (V/4) R  ->  multiply by i: (x, y) -> (-y, x)
    const double f = sp.w * kMu0 * G.vol * 0.25;
#pragma unroll
    for (int i = 0; i < 6; ++i) Rst[(size_t)i * T + t] = make_double2(-f * R[i].y, f * R[i].x);
}

// Receivers: one wavefront per receiver (the layered E_p), lane 0 adds the
// interpolated secondary field (eq. 8).
__global__ void __launch_bounds__(64)
k_receivers_layered(int n_rx, const double* __restrict__ rxyz, const int32_t* __restrict__ rtet,
                    const int32_t* __restrict__ rdof, const double* __restrict__ xyz, const int4* __restrict__ tets,
                    const double2* __restrict__ x, Layers L, LSrc sp, GL16 gl, double2* __restrict__ E,
                    double2* __restrict__ Es) {
    const int r = blockIdx.x;
    const double p[3] = {rxyz[3 * r], rxyz[3 * r + 1], rxyz[3 * r + 2]};
    double2 ep[3];
    layered_E(p, sp, L, gl, ep);
    if (threadIdx.x != 0) return;
    TetGeom G;
    tet_geometry(xyz, tets[rtet[r]], G);
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
        const int d = rdof[6 * r + i];
        if (d < 0) continue;
        const double2 v = x[d];
        const int a = kLE0[i], b = kLE1[i];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double nk = G.sl[i] * (lam[a] * G.g[b][k] - lam[b] * G.g[a][k]);
            es[k].x += nk * v.x;
            es[k].y += nk * v.y;
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        E[3 * r + k] = cadd(ep[k], es[k]);
        if (Es) Es[3 * r + k] = es[k];
    }
}

// Gauss-Legendre nodes and weights on [-1, 1]: Newton on P_16 from
// Chebyshev-like guesses, P_n and its derivative by the three-term recurrence.
GL16 make_gl16() {
    GL16 g;
    const int n = 16;
    for (int i = 0; i < n; ++i) {
        double x = std::cos(kPi * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
            const double step = p1 / dp;
            x -= step;
            if (std::fabs(step) < 1e-16) break;
        }
        g.x[i] = x;
        g.w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
    return g;
}

const GL16& gl16() {
    static const GL16 g = make_gl16();
    return g;
}

LSrc make_lsrc(const petgem_source& s) {
    LSrc p;
    for (int k = 0; k < 3; ++k) { p.pos[k] = s.pos[k]; p.dir[k] = s.dir[k]; }
    p.w = 2.0 * kPi * s.freq_hz;
    p.mom = s.moment;
    return p;
}

}  // namespace

int launch_rhs_layered(petgem_system* sys, const petgem_source& src, double2* Rst, int* flag, hipStream_t s) {
    if (!(src.pos[2] > sys->layers.z0)) {
        set_error("layered background: the source must lie above the interface");
        return PETGEM_INVALID_ARG;
    }
    hipLaunchKernelGGL(k_rhs_layered, dim3(sys->n_tets), dim3(64), 0, s, sys->n_tets, sys->xyz,
                       reinterpret_cast<const int4*>(sys->tets), sys->sigma, sys->layers, make_lsrc(src), gl16(),
                       1e-9 * sys->h_mean, Rst, flag);
    PG_HIP(hipGetLastError());
    return PETGEM_OK;
}

int launch_receivers_layered(const petgem_solution* sol, int k, int32_t n_rx, double2* E, double2* Es,
                             hipStream_t s) {
    const petgem_system* sys = sol->sys;
    hipLaunchKernelGGL(k_receivers_layered, dim3(n_rx), dim3(64), 0, s, n_rx, sys->rxc.xyz, sys->rxc.tet,
                       sys->rxc.dof, sys->xyz, reinterpret_cast<const int4*>(sys->tets),
                       sol->x + (size_t)k * sys->n_dof, sol->layers, make_lsrc(sol->src[k]), gl16(), E, Es);
    PG_HIP(hipGetLastError());
    return PETGEM_OK;
}

}  // namespace petgem
