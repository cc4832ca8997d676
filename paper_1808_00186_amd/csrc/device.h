// Device-side helpers for the gfx950 kernels: complex arithmetic on
// double2/float2, the XCD-aware block remap, wavefront reductions and the
// whole-space dipole field.
#pragma once
#include <hip/hip_runtime.h>

namespace petgem {

constexpr int kWave = 64;

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
    double d = 1.0 / (b.x * b.x + b.y * b.y);
    return make_double2((a.x * b.x + a.y * b.y) * d, (a.y * b.x - a.x * b.y) * d);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

// Workgroups are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b % 8). Remap so that each XCD works on one contiguous range of logical
// blocks: rows that share gathered x entries then share one L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
    int q = nb >> 3, r = nb & 7;
    int x = b & 7, i = b >> 3;
    return x * q + (x < r ? x : r) + i;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Primary field of a unit-direction dipole p with moment `mom` at src in a
// whole space of conductivity sigma (e^{-iwt}). With kappa = sqrt(w mu0 sigma/2)
// the wavenumber is k = (1+i) kappa, so e^{ikr} = e^{-kappa r} e^{i kappa r},
// (kr)^2 = 2i (kappa r)^2, and
//   E = mom/(4 pi sigma r^3) e^{ikr} [ d (d.p)/r^2 (3 - 3ikr - k^2 r^2)
//                                      + p (k^2 r^2 + ikr - 1) ].
__device__ __forceinline__ void dipole_E(const double x[3], const double src[3],
                                         const double p[3], double kappa, double pref,
                                         double2 E[3]) {
    double d0 = x[0] - src[0], d1 = x[1] - src[1], d2 = x[2] - src[2];
    double r2 = d0 * d0 + d1 * d1 + d2 * d2;
    double r = sqrt(r2);
    double kr = kappa * r;
    double s, c;
    sincos(kr, &s, &c);
    double a = pref * exp(-kr) / (r2 * r);
    double2 ph = make_double2(a * c, a * s);
    // A = 3 + 3 kr - i (3 kr + 2 kr^2);  B = -(1 + kr) + i (kr + 2 kr^2)
    double2 A = make_double2(3.0 + 3.0 * kr, -(3.0 * kr + 2.0 * kr * kr));
    double2 B = make_double2(-(1.0 + kr), kr + 2.0 * kr * kr);
    double dp = (d0 * p[0] + d1 * p[1] + d2 * p[2]) / r2;
    double2 Ad = cmul(ph, cscale(A, dp));
    double2 Bp = cmul(ph, B);
    E[0] = make_double2(Ad.x * d0 + Bp.x * p[0], Ad.y * d0 + Bp.y * p[0]);
    E[1] = make_double2(Ad.x * d1 + Bp.x * p[1], Ad.y * d1 + Bp.y * p[1]);
    E[2] = make_double2(Ad.x * d2 + Bp.x * p[2], Ad.y * d2 + Bp.y * p[2]);
}

// Primary magnetic field of the same dipole, H = curl E / (i w mu0)
// (Faraday's law with e^{-iwt}): the gradient part of E has no curl and
// k^2 = i w mu0 sigma, so H = mom grad G x p with G = e^{ikr} / (4 pi r),
//   H = mom (ikr - 1) e^{ikr} / (4 pi r^3) (d x p),
// and ikr - 1 = -(1 + kappa r) + i kappa r. hpref = mom / (4 pi).
__device__ __forceinline__ void dipole_H(const double x[3], const double src[3],
                                         const double p[3], double kappa, double hpref,
                                         double2 H[3]) {
    double d0 = x[0] - src[0], d1 = x[1] - src[1], d2 = x[2] - src[2];
    double r2 = d0 * d0 + d1 * d1 + d2 * d2;
    double r = sqrt(r2);
    double kr = kappa * r;
    double s, c;
    sincos(kr, &s, &c);
    double a = hpref * exp(-kr) / (r2 * r);
    const double2 f = cmul(make_double2(a * c, a * s), make_double2(-(1.0 + kr), kr));
    const double dxp[3] = {d1 * p[2] - d2 * p[1], d2 * p[0] - d0 * p[2], d0 * p[1] - d1 * p[0]};
#pragma unroll
    for (int k = 0; k < 3; ++k) H[k] = make_double2(f.x * dxp[k], f.y * dxp[k]);
}

// Barycentric gradients, volume, edge sign*length of a tetrahedron.
// J = [x1-x0, x2-x0, x3-x0]; grad lambda_{1,2,3} = rows of J^{-1}
// = (b x c, c x a, a x b)/det; grad lambda_0 = -sum.
struct TetGeom {
    double X[4][3];
    double g[4][3];
    double vol;
    double sl[6];   // s_i * l_i
};

__device__ __forceinline__ void tet_geometry(const double* __restrict__ xyz, int4 v, TetGeom& G) {
    const int id[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        G.X[k][0] = xyz[3 * (size_t)id[k] + 0];
        G.X[k][1] = xyz[3 * (size_t)id[k] + 1];
        G.X[k][2] = xyz[3 * (size_t)id[k] + 2];
    }
    double a[3], b[3], c[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        a[k] = G.X[1][k] - G.X[0][k];
        b[k] = G.X[2][k] - G.X[0][k];
        c[k] = G.X[3][k] - G.X[0][k];
    }
    double bc[3] = {b[1] * c[2] - b[2] * c[1], b[2] * c[0] - b[0] * c[2], b[0] * c[1] - b[1] * c[0]};
    double ca[3] = {c[1] * a[2] - c[2] * a[1], c[2] * a[0] - c[0] * a[2], c[0] * a[1] - c[1] * a[0]};
    double ab[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
    double det = a[0] * bc[0] + a[1] * bc[1] + a[2] * bc[2];
    double inv = 1.0 / det;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        G.g[1][k] = bc[k] * inv;
        G.g[2][k] = ca[k] * inv;
        G.g[3][k] = ab[k] * inv;
        G.g[0][k] = -(G.g[1][k] + G.g[2][k] + G.g[3][k]);
    }
    G.vol = fabs(det) * (1.0 / 6.0);
    constexpr int E0[6] = {0, 0, 0, 1, 3, 2};
    constexpr int E1[6] = {1, 2, 3, 2, 1, 3};
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        double dx = G.X[E1[i]][0] - G.X[E0[i]][0];
        double dy = G.X[E1[i]][1] - G.X[E0[i]][1];
        double dz = G.X[E1[i]][2] - G.X[E0[i]][2];
        double l = sqrt(dx * dx + dy * dy + dz * dz);
        G.sl[i] = (id[E1[i]] > id[E0[i]]) ? l : -l;
    }
}

}  // namespace petgem
