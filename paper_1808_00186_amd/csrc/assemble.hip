// Element matrices and deterministic global assembly (Section 3, eq. 9;
// Section 4; Appendix B, eqs. B.13-B.15).
//
// k_elem_km: one thread per tetrahedron computes the 21 unique entries of the
//   symmetric 6x6 curl-curl matrix K^e and of sigma_e M^e in closed form and
//   stores them structure-of-arrays ([21][T]) so that both the writes here and
//   the per-entry reads of the gather are coalesced in element order.
// k_gather: one thread per nonzero sums its element contributions in
//   increasing element order (fixed lists built on the host), so the assembled
//   values are bitwise reproducible and bitwise symmetric, without atomics.
#include "device.h"
#include "internal.h"

namespace petgem {

namespace {

constexpr int kE0[6] = {0, 0, 0, 1, 3, 2};
constexpr int kE1[6] = {1, 2, 3, 2, 1, 3};

__global__ void __launch_bounds__(256)
k_elem_km(int T, const double* __restrict__ xyz, const int4* __restrict__ tets,
          const double* __restrict__ sigma, double* __restrict__ Kst, double* __restrict__ Mst) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    TetGeom G;
    tet_geometry(xyz, tets[t], G);
    // curl N_i = 2 s_i l_i grad(lambda_a) x grad(lambda_b)
    double C[6][3];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        const double* ga = G.g[kE0[i]];
        const double* gb = G.g[kE1[i]];
        double f = 2.0 * G.sl[i];
        C[i][0] = f * (ga[1] * gb[2] - ga[2] * gb[1]);
        C[i][1] = f * (ga[2] * gb[0] - ga[0] * gb[2]);
        C[i][2] = f * (ga[0] * gb[1] - ga[1] * gb[0]);
    }
    // g_pq = grad lambda_p . grad lambda_q
    double gg[4][4];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = p; q < 4; ++q) {
            double v = G.g[p][0] * G.g[q][0] + G.g[p][1] * G.g[q][1] + G.g[p][2] * G.g[q][2];
            gg[p][q] = v;
            gg[q][p] = v;
        }
    const double V = G.vol;
    const double sV = sigma[t] * V * (1.0 / 20.0);
    int k = 0;
#pragma unroll
    for (int i = 0; i < 6; ++i) {
#pragma unroll
        for (int j = i; j < 6; ++j, ++k) {
            double kij = V * (C[i][0] * C[j][0] + C[i][1] * C[j][1] + C[i][2] * C[j][2]);
            // int lambda_p lambda_q = V (1 + delta_pq) / 20
            const int a = kE0[i], b = kE1[i], c = kE0[j], d = kE1[j];
            double m = (1.0 + (a == c)) * gg[b][d] - (1.0 + (a == d)) * gg[b][c]
                     - (1.0 + (b == c)) * gg[a][d] + (1.0 + (b == d)) * gg[a][c];
            Kst[(size_t)k * T + t] = kij;
            Mst[(size_t)k * T + t] = sV * G.sl[i] * G.sl[j] * m;
        }
    }
}

__global__ void __launch_bounds__(256)
k_gather(int64_t nnz, const int32_t* __restrict__ cptr, const int32_t* __restrict__ cidx,
         const double* __restrict__ Kst, const double* __restrict__ Mst,
         double* __restrict__ K, double* __restrict__ Ms) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nnz) return;
    double sk = 0.0, sm = 0.0;
    const int32_t c1 = cptr[k + 1];
    // four contribution indices, then their values, in flight at a time; the
    // sums keep the list order
    for (int32_t c = cptr[k]; c < c1; c += 4) {
        int32_t idx[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) idx[q] = c + q < c1 ? cidx[c + q] : -1;
        double kv[4], mv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            kv[q] = idx[q] >= 0 ? Kst[idx[q]] : 0.0;
            mv[q] = idx[q] >= 0 ? Mst[idx[q]] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (idx[q] >= 0) {
                sk += kv[q];
                sm += mv[q];
            }
    }
    K[k] = sk;
    Ms[k] = sm;
}

__global__ void k_diag(int n, const int32_t* __restrict__ dpos, const double* __restrict__ K,
                       const double* __restrict__ Ms, double* __restrict__ Kd, double* __restrict__ Msd) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    Kd[r] = K[dpos[r]];
    Msd[r] = Ms[dpos[r]];
}

// D = diag(A) = Kd - i w mu0 Msd and its inverse.
__global__ void k_jacobi(int n, double wmu, const double* __restrict__ Kd,
                         const double* __restrict__ Msd, double2* __restrict__ dvec,
                         double2* __restrict__ dinv) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    double2 d = make_double2(Kd[r], -wmu * Msd[r]);
    dvec[r] = d;
    dinv[r] = cdiv(make_double2(1.0, 0.0), d);
}

// Ahat_k = (K_k - i w mu0 Ms_k) / D_col(k): the right-Jacobi-preconditioned
// operator A D^{-1} of the double-precision GMRES.
__global__ void __launch_bounds__(256)
k_ahat(int n, double wmu, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
       const double* __restrict__ K, const double* __restrict__ Ms,
       const double2* __restrict__ dinv, double2* __restrict__ Ahat) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    for (int32_t k = rp[r]; k < rp[r + 1]; ++k)
        Ahat[k] = cmul(make_double2(K[k], -wmu * Ms[k]), dinv[col[k]]);
}

__global__ void k_to_f32(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
                         float* __restrict__ a32, float* __restrict__ b32) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    a32[i] = (float)a[i];
    b32[i] = (float)b[i];
}

}  // namespace

int launch_assembly(petgem_system* sys, hipStream_t s) {
    const int T = sys->n_tets;
    hipLaunchKernelGGL(k_elem_km, dim3(ceil_div(T, 256)), dim3(256), 0, s, T, sys->xyz,
                       reinterpret_cast<const int4*>(sys->tets), sys->sigma, sys->Kst, sys->Mst);
    PG_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_gather, dim3(ceil_div(sys->nnz, 256)), dim3(256), 0, s, sys->nnz,
                       sys->cptr, sys->cidx, sys->Kst, sys->Mst, sys->K, sys->Ms);
    PG_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_diag, dim3(ceil_div(sys->n_dof, 256)), dim3(256), 0, s, sys->n_dof,
                       sys->diag_pos, sys->K, sys->Ms, sys->Kd, sys->Msd);
    PG_HIP(hipGetLastError());
    sys->cached_freq = -1.0;   // operators derived from K, Ms are stale
    sys->have32 = false;
    return PETGEM_OK;
}

int launch_freq_prep(petgem_system* sys, double freq, hipStream_t s) {
    if (sys->cached_freq == freq) return PETGEM_OK;
    const int n = sys->n_dof;
    if (!sys->Ahat) {
        PG_TRY(dalloc(&sys->Ahat, sys->nnz));
        PG_TRY(dalloc(&sys->dvec, n));
        PG_TRY(dalloc(&sys->dinv, n));
    }
    const double wmu = 2.0 * kPi * freq * kMu0;
    hipLaunchKernelGGL(k_jacobi, dim3(ceil_div(n, 256)), dim3(256), 0, s, n, wmu, sys->Kd,
                       sys->Msd, sys->dvec, sys->dinv);
    hipLaunchKernelGGL(k_ahat, dim3(ceil_div(n, 256)), dim3(256), 0, s, n, wmu, sys->row_ptr,
                       sys->col, sys->K, sys->Ms, sys->dinv, sys->Ahat);
    PG_HIP(hipGetLastError());
    sys->cached_freq = freq;
    return PETGEM_OK;
}

int ensure_fp32(petgem_system* sys, hipStream_t s) {
    if (sys->have32) return PETGEM_OK;
    if (!sys->K32) {
        PG_TRY(dalloc(&sys->K32, sys->nnz));
        PG_TRY(dalloc(&sys->Ms32, sys->nnz));
    }
    hipLaunchKernelGGL(k_to_f32, dim3(ceil_div(sys->nnz, 256)), dim3(256), 0, s, sys->nnz, sys->K,
                       sys->Ms, sys->K32, sys->Ms32);
    PG_HIP(hipGetLastError());
    sys->have32 = true;
    sys->sell32.values = false;
    sys->ssor32.values = false;
    return PETGEM_OK;
}

}  // namespace petgem
