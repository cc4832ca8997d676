// Double-precision right-Jacobi-preconditioned restarted GMRES on the GPU
// (the paper solves its systems with PETSc GMRES, Section 5.1).
//
// The operator is Ahat = A D^{-1} (D = diag A), stored as complex128 CSR, so
// the residual of the iterate u = D x is the true residual b - A x. One
// Arnoldi step is four kernels:
//   k_spmv   w = Ahat v_j                       (CSR, G lanes per row)
//   k_mdot   partial sums of v_k^H w (k <= j) and |w|^2, fixed block split
//   k_fin    one workgroup: fixed-order reduction, Hessenberg column, the
//            Givens update of the least-squares residual, convergence flag
//   k_update v_{j+1} = (w - sum_k h_k v_k) / beta
// Classical Gram-Schmidt with the norm from Pythagoras costs one pass over
// the basis for the dots and one for the update; when cancellation makes the
// Pythagorean norm unreliable (beta^2 <= eta |w|^2) the step requests a
// second Gram-Schmidt pass, whose kernels otherwise exit at once. All
// reductions use a fixed partition and order, so the solve is bitwise
// reproducible. Every kernel reads the cycle's `done` flag and returns early
// once the estimate has converged, which lets a whole cycle be captured in a
// HIP graph and replayed without host round trips; the host reads back one
// small record per cycle, after the true residual has been recomputed.
#include <array>
#include <chrono>
#include <cstddef>
#include <cstdio>
#include <utility>

#include <hip/hip_ext.h>

#include "device.h"
#include "internal.h"

namespace petgem {

namespace {

constexpr int kDotMaxBlocks = 1024;
constexpr int kChunk = 16;        // coefficients accumulated per pass of k_mdot
constexpr double kEta = 1e-2;     // re-orthogonalise when beta^2 <= eta |w|^2

// y = Ahat x, or y = b - Ahat x when RES. G lanes cooperate on one row.
template <int G, bool RES>
__global__ void __launch_bounds__(256)
k_spmv(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
       const double2* __restrict__ val, const double2* __restrict__ x,
       const double2* __restrict__ b, double2* __restrict__ y, const int* __restrict__ done) {
    if (done && *done) return;
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int row = (blk * 256 + (int)threadIdx.x) / G;
    const int lane = threadIdx.x & (G - 1);
    if (row >= n) return;
    double2 acc = make_double2(0.0, 0.0);
    const int32_t e = rp[row + 1];
    // 2 nonzeros per lane in flight
    for (int32_t k0 = rp[row] + lane; k0 < e; k0 += 2 * G) {
        const int32_t k1 = k0 + G;
        const int32_t c0 = col[k0];
        const int32_t c1 = k1 < e ? col[k1] : -1;
        const double2 a0 = val[k0];
        const double2 a1 = k1 < e ? val[k1] : make_double2(0.0, 0.0);
        const double2 v0 = x[c0];
        const double2 v1 = c1 >= 0 ? x[c1] : make_double2(0.0, 0.0);
        acc.x += a0.x * v0.x - a0.y * v0.y;
        acc.y += a0.x * v0.y + a0.y * v0.x;
        acc.x += a1.x * v1.x - a1.y * v1.y;
        acc.y += a1.x * v1.y + a1.y * v1.x;
    }
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) {
        acc.x += __shfl_xor(acc.x, off, G);
        acc.y += __shfl_xor(acc.y, off, G);
    }
    if (lane == 0) y[row] = RES ? csub(b[row], acc) : acc;
}

// partial[k][blk] = sum_i conj(V_k[i]) w[i] (k <= j), partial[j+1][blk] = sum |w_i|^2.
// flags: 0 = unconditional, 1 = skip when done, 2 = skip when done or !reorth.
__global__ void __launch_bounds__(256)
k_mdot(int n, int j, const double2* __restrict__ V, size_t ldv, const double2* __restrict__ w,
       double2* __restrict__ partial, const GmresCtl* __restrict__ ctl, int flags) {
    if (flags >= 1 && ctl->done) return;
    if (flags == 2 && !ctl->reorth) return;
    __shared__ double2 red[4][kChunk];
    const int nb = gridDim.x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int c0 = 0; c0 <= j + 1; c0 += kChunk) {
        double2 acc[kChunk];
#pragma unroll
        for (int q = 0; q < kChunk; ++q) acc[q] = make_double2(0.0, 0.0);
        for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += nb * 256) {
            const double2 wi = w[i];
#pragma unroll
            for (int q = 0; q < kChunk; ++q) {
                const int k = c0 + q;
                if (k <= j) {
                    const double2 v = V[(size_t)k * ldv + i];
                    acc[q].x += v.x * wi.x + v.y * wi.y;
                    acc[q].y += v.x * wi.y - v.y * wi.x;
                } else if (k == j + 1) {
                    acc[q].x += wi.x * wi.x + wi.y * wi.y;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < kChunk; ++q) {
            double rx = wave_sum(acc[q].x), ry = wave_sum(acc[q].y);
            if (lane == 0) red[wave][q] = make_double2(rx, ry);
        }
        __syncthreads();
        if (threadIdx.x < kChunk && c0 + (int)threadIdx.x <= j + 1) {
            const int q = threadIdx.x;
            double2 s = red[0][q];
            s = cadd(s, red[1][q]);
            s = cadd(s, red[2][q]);
            s = cadd(s, red[3][q]);
            partial[(size_t)(c0 + q) * nb + blockIdx.x] = s;
        }
        __syncthreads();
    }
}

// Same as k_mdot with the number of dot products fixed at compile time
// (NK = j + 1, plus |w|^2): straight-line loads of all basis vectors of a row.
template <int NK>
__global__ void __launch_bounds__(256)
k_mdot_t(int n, const double2* __restrict__ V, size_t ldv, const double2* __restrict__ w,
         double2* __restrict__ partial, const GmresCtl* __restrict__ ctl, int flags) {
    if (flags >= 1 && ctl->done) return;
    if (flags == 2 && !ctl->reorth) return;
    __shared__ double2 red[4][NK + 1];
    const int nb = gridDim.x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double2 acc[NK];
    double nrm = 0.0;
#pragma unroll
    for (int q = 0; q < NK; ++q) acc[q] = make_double2(0.0, 0.0);
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += nb * 256) {
        const double2 wi = w[i];
        double2 v[NK];
#pragma unroll
        for (int q = 0; q < NK; ++q) v[q] = V[(size_t)q * ldv + i];
#pragma unroll
        for (int q = 0; q < NK; ++q) {
            acc[q].x += v[q].x * wi.x + v[q].y * wi.y;
            acc[q].y += v[q].x * wi.y - v[q].y * wi.x;
        }
        nrm += wi.x * wi.x + wi.y * wi.y;
    }
#pragma unroll
    for (int q = 0; q < NK; ++q) {
        const double rx = wave_sum(acc[q].x), ry = wave_sum(acc[q].y);
        if (lane == 0) red[wave][q] = make_double2(rx, ry);
    }
    nrm = wave_sum(nrm);
    if (lane == 0) red[wave][NK] = make_double2(nrm, 0.0);
    __syncthreads();
    for (int q = threadIdx.x; q <= NK; q += blockDim.x) {
        double2 s = red[0][q];
        s = cadd(s, red[1][q]);
        s = cadd(s, red[2][q]);
        s = cadd(s, red[3][q]);
        partial[(size_t)q * nb + blockIdx.x] = s;
    }
}

// Fixed-order sum of the block partials of coefficients 0..kmax into coef[]
// (nb <= 1024: every lane issues its up to 16 loads before summing).
__device__ void reduce_partials(int kmax, int nb, const double2* __restrict__ partial, double2* coef) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nw = blockDim.x >> 6;
    for (int k = wave; k <= kmax; k += nw) {
        double2 p[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int b = lane + 64 * u;
            p[u] = b < nb ? partial[(size_t)k * nb + b] : make_double2(0.0, 0.0);
        }
        double sx = 0.0, sy = 0.0;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            sx += p[u].x;
            sy += p[u].y;
        }
        sx = wave_sum(sx);
        sy = wave_sum(sy);
        if (lane == 0) coef[k] = make_double2(sx, sy);
    }
    __syncthreads();
}

__device__ __forceinline__ double2& Hij(GmresCtl* c, int i, int j) { return c->H[j * (kMaxRestart + 1) + i]; }

// One workgroup: finish the Gram-Schmidt pass of Arnoldi step j. The
// Hessenberg column, the previous rotations and g are staged in LDS so that
// the sequential Givens recurrence runs on LDS, not on global memory.
__global__ void __launch_bounds__(1024)
k_fin(int j, int nb, const double2* __restrict__ partial, GmresCtl* __restrict__ ctl, int pass) {
    if (ctl->done) return;
    if (pass == 1 && !ctl->reorth) return;
    __shared__ double2 coef[kMaxRestart + 2];
    __shared__ double2 col[kMaxRestart + 2];
    __shared__ double2 rc[kMaxRestart], rs[kMaxRestart];
    __shared__ int accept;
    GmresCtl* c = ctl;
    reduce_partials(j + 1, nb, partial, coef);   // ends with __syncthreads
    const int t = threadIdx.x;
    if (t <= j) {
        col[t] = pass == 0 ? coef[t] : cadd(Hij(c, t, j), coef[t]);
        c->h[t] = coef[t];
    }
    if (t < j) {
        rc[t] = c->cs[t];
        rs[t] = c->sn[t];
    }
    __syncthreads();
    if (t == 0) {
        accept = 0;
        const double nrm2 = coef[j + 1].x;
        double hh = 0.0;
        for (int k = 0; k <= j; ++k) hh += cabs2(coef[k]);
        if (!isfinite(nrm2) || !isfinite(hh)) {
            c->nonfinite = 1;
            c->done = 1;
        } else if (pass == 0 && nrm2 - hh <= kEta * nrm2) {   // cancellation: second pass
            c->reorth = 1;
            c->scale = 1.0;
            accept = 2;   // store the unrotated column for the second pass
        } else {
            const double beta2 = nrm2 - hh;
            c->reorth = pass;   // pass 1 keeps the flag so that its update runs
            const double beta = beta2 > 0.0 ? sqrt(beta2) : 0.0;
            c->scale = beta > 0.0 ? 1.0 / beta : 0.0;
            // previous rotations [[conj(c), conj(s)], [-s, c]] on rows (i, i+1)
            for (int i = 0; i < j; ++i) {
                const double2 a = col[i], b = col[i + 1];
                col[i] = cadd(cmulc(rc[i], a), cmulc(rs[i], b));
                col[i + 1] = csub(cmul(rc[i], b), cmul(rs[i], a));
            }
            const double2 a = col[j];
            const double den = sqrt(cabs2(a) + beta * beta);
            double2 cs, sn;
            if (den > 0.0) {
                cs = cscale(a, 1.0 / den);
                sn = make_double2(beta / den, 0.0);
            } else {
                cs = make_double2(1.0, 0.0);
                sn = make_double2(0.0, 0.0);
            }
            c->cs[j] = cs;
            c->sn[j] = sn;
            col[j] = make_double2(den, 0.0);
            col[j + 1] = make_double2(0.0, 0.0);
            const double2 gj = c->g[j];
            const double2 g1 = cscale(cmul(sn, gj), -1.0);
            c->g[j + 1] = g1;
            c->g[j] = cmulc(cs, gj);
            c->mdone = j + 1;
            if (sqrt(cabs2(g1)) <= c->tol_abs || beta <= 1e-300) c->done = 1;
            accept = 1;
        }
    }
    __syncthreads();
    if (accept && t <= j + 1) {
        if (accept == 1 || t <= j) Hij(c, t, j) = col[t];
    }
}

// v_{j+1} = (w - sum_k h_k v_k) * scale, in place in slot j+1.
__global__ void __launch_bounds__(256)
k_update(int n, int j, double2* __restrict__ V, size_t ldv, const GmresCtl* __restrict__ ctl, int pass) {
    if (ctl->done) return;
    if (pass == 1 && !ctl->reorth) return;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double2 w = V[(size_t)(j + 1) * ldv + i];
    for (int k = 0; k <= j; ++k) {
        const double2 h = ctl->h[k];
        const double2 v = V[(size_t)k * ldv + i];
        w.x -= h.x * v.x - h.y * v.y;
        w.y -= h.x * v.y + h.y * v.x;
    }
    const double s = ctl->scale;
    V[(size_t)(j + 1) * ldv + i] = make_double2(w.x * s, w.y * s);
}

// Back substitution R y = g over the completed steps; R and g are staged in
// LDS by the whole workgroup, the recurrence runs on one thread.
__global__ void __launch_bounds__(256) k_trisolve(GmresCtl* __restrict__ c) {
    __shared__ double2 R[kMaxRestart * kMaxRestart];
    __shared__ double2 y[kMaxRestart];
    const int m = c->mdone;
    for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
        const int i = e % m, k = e / m;
        if (i <= k) R[k * kMaxRestart + i] = Hij(c, i, k);
    }
    if ((int)threadIdx.x < m) y[threadIdx.x] = c->g[threadIdx.x];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = m - 1; i >= 0; --i) {
            double2 s = y[i];
            for (int k = i + 1; k < m; ++k) s = csub(s, cmul(R[k * kMaxRestart + i], y[k]));
            y[i] = cdiv(s, R[i * kMaxRestart + i]);
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < m) c->y[threadIdx.x] = y[threadIdx.x];
}

// u += sum_{k < mdone} y_k v_k
__global__ void __launch_bounds__(256)
k_xupdate(int n, const double2* __restrict__ V, size_t ldv, double2* __restrict__ u,
          const GmresCtl* __restrict__ ctl) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int m = ctl->mdone;
    double2 acc = u[i];
    for (int k = 0; k < m; ++k) acc = cadd(acc, cmul(ctl->y[k], V[(size_t)k * ldv + i]));
    u[i] = acc;
}

// Start of a cycle: rnorm = |r| from the partials, g = (rnorm, 0, ...).
struct CycleTail {   // mirrored to the host once per cycle
    double rnorm;
    int last_m;
    int nonfinite;
};

__global__ void __launch_bounds__(1024)
k_cycle_start(int nb, const double2* __restrict__ partial, GmresCtl* __restrict__ c,
              CycleTail* __restrict__ tail) {
    __shared__ double2 coef[2];
    reduce_partials(0, nb, partial, coef);
    if (threadIdx.x != 0) return;
    const double r2 = coef[0].x;
    const double rn = sqrt(r2);
    tail->rnorm = rn;
    tail->last_m = c->mdone;
    tail->nonfinite = c->nonfinite || !isfinite(r2);
    c->rnorm = rn;
    c->scale = rn > 0.0 ? 1.0 / rn : 0.0;
    c->g[0] = make_double2(rn, 0.0);
    c->done = (rn <= c->tol_abs || !isfinite(r2)) ? 1 : 0;
    c->mdone = 0;
    c->reorth = 0;
    c->nonfinite = 0;
}

__global__ void k_scale_v0(int n, double2* __restrict__ v, const GmresCtl* __restrict__ c) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    v[i] = cscale(v[i], c->scale);
}

__global__ void k_set_tol(GmresCtl* c, double tol) {
    c->tol_abs = tol;
    c->done = 0;
    c->mdone = 0;
    c->reorth = 0;
    c->nonfinite = 0;
}

__global__ void k_fill0(int n, double2* __restrict__ u) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) u[i] = make_double2(0.0, 0.0);
}

// u = D x0 (scaled iterate of a caller-supplied guess)
__global__ void k_scale_in(int n, const double2* __restrict__ d, const double2* __restrict__ x,
                           double2* __restrict__ u) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) u[i] = cmul(d[i], x[i]);
}

// Minimal-residual scaling of a supplied guess: partials of w^H b and |w|^2
// for w = A x0 (fixed block split).
__global__ void __launch_bounds__(256)
k_dots_wb(int n, const double2* __restrict__ w, const double2* __restrict__ b, double2* __restrict__ partial) {
    __shared__ double2 red[4][2];
    const int nb = gridDim.x, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double2 wb = make_double2(0.0, 0.0);
    double ww = 0.0;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += nb * 256) {
        const double2 wi = w[i], bi = b[i];
        wb = cadd(wb, cmulc(wi, bi));
        ww += cabs2(wi);
    }
    wb.x = wave_sum(wb.x);
    wb.y = wave_sum(wb.y);
    ww = wave_sum(ww);
    if (lane == 0) { red[wave][0] = wb; red[wave][1] = make_double2(ww, 0.0); }
    __syncthreads();
    if (threadIdx.x < 2) {
        double2 t = red[0][threadIdx.x];
        t = cadd(t, red[1][threadIdx.x]);
        t = cadd(t, red[2][threadIdx.x]);
        t = cadd(t, red[3][threadIdx.x]);
        partial[(size_t)threadIdx.x * nb + blockIdx.x] = t;
    }
}

// u *= alpha with alpha = (w^H b) / |w|^2 (0 when w vanishes or is not finite)
__global__ void __launch_bounds__(1024) k_x0_alpha(int nb, const double2* __restrict__ partial, double2* __restrict__ alpha) {
    __shared__ double2 coef[2];
    reduce_partials(1, nb, partial, coef);
    if (threadIdx.x != 0) return;
    const double2 wb = coef[0];
    const double ww = coef[1].x;
    double2 a = make_double2(0.0, 0.0);
    if (ww > 0.0 && isfinite(ww) && isfinite(wb.x) && isfinite(wb.y)) a = cscale(wb, 1.0 / ww);
    *alpha = a;
}

__global__ void k_scale_by(int n, const double2* __restrict__ alpha, double2* __restrict__ u) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) u[i] = cmul(*alpha, u[i]);
}

}  // namespace

void GmresWork::release() {
    if (graph) (void)hipGraphExecDestroy(graph);
    graph = nullptr;
    if (graph_stream) (void)hipStreamDestroy(graph_stream);
    graph_stream = nullptr;
    dfree(V); dfree(u); dfree(b); dfree(partial); dfree(ctl);
    if (ctl_host) (void)hipHostFree(ctl_host);
    ctl_host = nullptr;
    n = m = nb_dot = 0;
}

namespace {

template <int... I>
constexpr auto mdot_table(std::integer_sequence<int, I...>) {
    using Fn = void (*)(int, const double2*, size_t, const double2*, double2*, const GmresCtl*, int);
    return std::array<Fn, sizeof...(I)>{&k_mdot_t<I + 1>...};
}
constexpr int kMdotT = 32;
const auto kMdotFns = mdot_table(std::make_integer_sequence<int, kMdotT>{});

// Dots of w with v_0..v_j (and |w|^2) into `partial`; j = -1 gives |w|^2 only.
void mdot_launch(int j, int nb, int n, const double2* V, size_t ldv, const double2* w,
                 double2* partial, const GmresCtl* ctl, int flags, hipStream_t s) {
    if (j >= 0 && j < kMdotT)
        hipLaunchKernelGGL(kMdotFns[j], dim3(nb), dim3(256), 0, s, n, V, ldv, w, partial, ctl, flags);
    else
        hipLaunchKernelGGL(k_mdot, dim3(nb), dim3(256), 0, s, n, j, V, ldv, w, partial, ctl, flags);
}

// e0 / e1 (optional): events the dispatch itself timestamps at the kernel's
// start and end, for profiling without extra packets between kernels.
template <bool RES>
void spmv_launch(int G, int n, const int32_t* rp, const int32_t* col, const double2* val,
                 const double2* x, const double2* b, double2* y, const int* done, hipStream_t s,
                 hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
    const int nblk = ceil_div((int64_t)n * G, 256);
    auto go = [&](auto kernel) {   // the timestamping dispatch only when profiling
        if (e0)
            hipExtLaunchKernelGGL(kernel, dim3(nblk), dim3(256), 0, s, e0, e1, 0, n, rp, col, val, x, b, y, done);
        else
            hipLaunchKernelGGL(kernel, dim3(nblk), dim3(256), 0, s, n, rp, col, val, x, b, y, done);
    };
    switch (G) {
        case 4: go(k_spmv<4, RES>); break;
        case 16: go(k_spmv<16, RES>); break;
        default: go(k_spmv<8, RES>); break;
    }
}

int ensure_gmres_work(petgem_system* sys, int m) {
    GmresWork& w = sys->gw;
    const int n = sys->n_dof;
    if (w.n == n && w.m == m) return PETGEM_OK;
    w.release();
    w.n = n;
    w.m = m;
    w.nb_dot = std::min(kDotMaxBlocks, ceil_div(n, 256));
    PG_TRY(dalloc(&w.V, (size_t)(m + 1) * n));
    PG_TRY(dalloc(&w.u, (size_t)n));
    PG_TRY(dalloc(&w.b, (size_t)n));
    PG_TRY(dalloc(&w.partial, (size_t)2 * (m + 2) * w.nb_dot + 16));
    PG_TRY(dalloc(&w.ctl, 1));
    PG_HIP(hipHostMalloc(reinterpret_cast<void**>(&w.ctl_host), sizeof(GmresCtl) + 64));
    return PETGEM_OK;
}

struct Timer {
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    double ms() const {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
};

// Profiling: a pair of events per sparse-matrix launch, timestamped by the
// dispatch itself (start and end of the kernel).
struct SpmvTimer {
    bool on = false;
    std::vector<hipEvent_t> ev;
    // the (start, end) events for the next launch, or nulls when off
    std::pair<hipEvent_t, hipEvent_t> next() {
        if (!on) return {nullptr, nullptr};
        hipEvent_t a, b;
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
        ev.push_back(a);
        ev.push_back(b);
        return {a, b};
    }
    void collect(petgem_stats* st) {
        if (!on) return;
        (void)hipEventSynchronize(ev.empty() ? nullptr : ev.back());
        double tot = 0.0;
        for (size_t i = 0; i + 1 < ev.size(); i += 2) {
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, ev[i], ev[i + 1]);
            tot += ms;
        }
        if (st) {
            st->spmv_ms += tot;
            st->spmv_launches += int(ev.size() / 2);
        }
        for (auto e : ev) (void)hipEventDestroy(e);
        ev.clear();
    }
};

}  // namespace

// Autotuner of the double-precision CSR SpMV: times the 4-, 8- and 16-lane
// row groups on this system's operator (5 launches each, HIP events on the
// caller's stream) and keeps the fastest. The choice is made once per system,
// so every solve on a system uses one summation order (bitwise reproducible
// within the system's lifetime).
int tune_spmv(petgem_system* sys, hipStream_t s) {
    if (sys->spmv_tuned) return PETGEM_OK;
    const int n = sys->n_dof;
    double2 *x = nullptr, *y = nullptr;
    PG_TRY(dalloc(&x, (size_t)n));
    PG_TRY(dalloc(&y, (size_t)n));
    hipLaunchKernelGGL(k_fill0, dim3(ceil_div(n, 256)), dim3(256), 0, s, n, x);
    hipEvent_t e0, e1;
    PG_HIP(hipEventCreate(&e0));
    PG_HIP(hipEventCreate(&e1));
    float best = 1e30f;
    int bestG = 8;
    for (int G : {4, 8, 16}) {
        spmv_launch<false>(G, n, sys->row_ptr, sys->col, sys->Ahat, x, nullptr, y, nullptr, s);  // warm
        PG_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < 5; ++r)
            spmv_launch<false>(G, n, sys->row_ptr, sys->col, sys->Ahat, x, nullptr, y, nullptr, s);
        PG_HIP(hipEventRecord(e1, s));
        PG_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        PG_HIP(hipEventElapsedTime(&ms, e0, e1));
        sys->spmv_tune_ms[G == 4 ? 0 : (G == 8 ? 1 : 2)] = ms / 5.0f;
        if (ms < best) { best = ms; bestG = G; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    dfree(x);
    dfree(y);
    sys->spmv_group = bestG;
    sys->spmv_tuned = true;
    return PETGEM_OK;
}

int launch_spmv_ahat(petgem_system* sys, const double2* x, double2* y, hipStream_t s) {
    spmv_launch<false>(sys->spmv_group, sys->n_dof, sys->row_ptr, sys->col, sys->Ahat, x, nullptr, y,
                       nullptr, s);
    PG_HIP(hipGetLastError());
    return PETGEM_OK;
}

int launch_spmv_unscaled(petgem_system* sys, const double2* x, double2* y, hipStream_t s) {
    const int n = sys->n_dof;
    if (!sys->tmp) PG_TRY(dalloc(&sys->tmp, (size_t)n));
    hipLaunchKernelGGL(k_scale_in, dim3(ceil_div(n, 256)), dim3(256), 0, s, n, sys->dvec, x, sys->tmp);
    return launch_spmv_ahat(sys, sys->tmp, y, s);
}

int gmres_solve(petgem_system* sys, const petgem_source& src, const petgem_opts& o,
                const double2* x0, double2* x_out, hipStream_t s, petgem_stats* st) {
    const int n = sys->n_dof;
    const int m = o.restart;
    Timer t_all;
    PG_TRY(launch_freq_prep(sys, src.freq_hz, s));
    PG_TRY(tune_spmv(sys, s));
    PG_TRY(ensure_gmres_work(sys, m));
    GmresWork& w = sys->gw;
    const int G = sys->spmv_group;
    const int nbv = ceil_div(n, 256);
    const size_t ldv = (size_t)n;
    CycleTail* tail = reinterpret_cast<CycleTail*>(reinterpret_cast<char*>(w.ctl_host) + sizeof(GmresCtl));
    CycleTail* tail_d = reinterpret_cast<CycleTail*>(reinterpret_cast<char*>(w.partial) +
                                                     sizeof(double2) * (size_t)(m + 2) * w.nb_dot);
    SpmvTimer prof;
    prof.on = o.profile != 0;

    // right-hand side
    Timer t_rhs;
    PG_TRY(launch_rhs(sys, src, w.b, 1, s));
    if (st) st->t_rhs_ms = t_rhs.ms();

    auto residual = [&]() -> int {   // V0 = b - Ahat u, rnorm, g, flags
        const auto pe = prof.next();
        spmv_launch<true>(G, n, sys->row_ptr, sys->col, sys->Ahat, w.u, w.b, w.V, nullptr, s, pe.first,
                          pe.second);
        mdot_launch(-1, w.nb_dot, n, w.V, ldv, w.V, reinterpret_cast<double2*>(w.partial), w.ctl, 0, s);
        hipLaunchKernelGGL(k_cycle_start, dim3(1), dim3(1024), 0, s, w.nb_dot,
                           reinterpret_cast<const double2*>(w.partial), w.ctl, tail_d);
        hipLaunchKernelGGL(k_scale_v0, dim3(nbv), dim3(256), 0, s, n, w.V, w.ctl);
        PG_HIP(hipGetLastError());
        return PETGEM_OK;
    };
    auto read_tail = [&]() -> int {
        PG_HIP(hipMemcpyAsync(tail, tail_d, sizeof(CycleTail), hipMemcpyDeviceToHost, s));
        PG_HIP(hipStreamSynchronize(s));
        return PETGEM_OK;
    };
    auto cycle = [&]() -> int {
        double2* part = reinterpret_cast<double2*>(w.partial);
        for (int j = 0; j < m; ++j) {
            double2* vj = w.V + (size_t)j * ldv;
            double2* vj1 = w.V + (size_t)(j + 1) * ldv;
            const auto pe = prof.next();
            spmv_launch<false>(G, n, sys->row_ptr, sys->col, sys->Ahat, vj, nullptr, vj1, &w.ctl->done, s,
                               pe.first, pe.second);
            mdot_launch(j, w.nb_dot, n, w.V, ldv, vj1, part, w.ctl, 1, s);
            hipLaunchKernelGGL(k_fin, dim3(1), dim3(1024), 0, s, j, w.nb_dot, part, w.ctl, 0);
            hipLaunchKernelGGL(k_update, dim3(nbv), dim3(256), 0, s, n, j, w.V, ldv, w.ctl, 0);
            mdot_launch(j, w.nb_dot, n, w.V, ldv, vj1, part, w.ctl, 2, s);
            hipLaunchKernelGGL(k_fin, dim3(1), dim3(1024), 0, s, j, w.nb_dot, part, w.ctl, 1);
            hipLaunchKernelGGL(k_update, dim3(nbv), dim3(256), 0, s, n, j, w.V, ldv, w.ctl, 1);
        }
        hipLaunchKernelGGL(k_trisolve, dim3(1), dim3(256), 0, s, w.ctl);
        hipLaunchKernelGGL(k_xupdate, dim3(nbv), dim3(256), 0, s, n, w.V, ldv, w.u, w.ctl);
        PG_HIP(hipGetLastError());
        return residual();
    };

    // |b| via the residual of u = 0
    hipLaunchKernelGGL(k_set_tol, dim3(1), dim3(1), 0, s, w.ctl, 0.0);
    hipLaunchKernelGGL(k_fill0, dim3(nbv), dim3(256), 0, s, n, w.u);
    PG_TRY(residual());
    PG_TRY(read_tail());
    int flag_h = 0;
    PG_HIP(hipMemcpy(&flag_h, sys->dflag, sizeof(int), hipMemcpyDeviceToHost));
    if (flag_h) {
        int zero = 0;
        PG_HIP(hipMemcpy(sys->dflag, &zero, sizeof(int), hipMemcpyHostToDevice));
        set_error("source within 1e-9 h of a quadrature point of an element with dsigma != 0");
        return PETGEM_SOURCE_SINGULAR;
    }
    const double bnorm = tail->rnorm;
    if (st) {
        st->b_norm = bnorm;
        st->iters = 0;
        st->ir_steps = 0;
        st->used_fallback = 0;
        st->x0_rel_residual = 1.0;
    }
    if (tail->nonfinite) {
        set_error("non-finite right-hand side");
        if (st) st->status = PETGEM_NONFINITE;
        return PETGEM_NONFINITE;
    }
    if (bnorm == 0.0) {
        hipLaunchKernelGGL(k_fill0, dim3(nbv), dim3(256), 0, s, n, x_out);
        if (st) { st->rel_residual = 0.0; st->status = PETGEM_OK; st->t_solve_ms = t_all.ms(); }
        return PETGEM_OK;
    }
    const double tol_abs = o.rtol * bnorm;
    double rnorm = bnorm;
    if (x0) {
        hipLaunchKernelGGL(k_scale_in, dim3(nbv), dim3(256), 0, s, n, sys->dvec, x0, w.u);
        // scale the guess by the alpha minimising |b - alpha A x0| (w = A x0 in slot 1)
        double2* wv = w.V + ldv;
        double2* part = reinterpret_cast<double2*>(w.partial);
        spmv_launch<false>(G, n, sys->row_ptr, sys->col, sys->Ahat, w.u, nullptr, wv, nullptr, s);
        hipLaunchKernelGGL(k_dots_wb, dim3(w.nb_dot), dim3(256), 0, s, n, wv, w.b, part);
        // one scalar in the slack after the partial sums and the cycle record
        double2* alpha = reinterpret_cast<double2*>(w.partial) + (size_t)(m + 2) * w.nb_dot + 4;
        hipLaunchKernelGGL(k_x0_alpha, dim3(1), dim3(1024), 0, s, w.nb_dot, part, alpha);
        hipLaunchKernelGGL(k_scale_by, dim3(nbv), dim3(256), 0, s, n, alpha, w.u);
        PG_TRY(residual());
        PG_TRY(read_tail());
        const double r0 = tail->rnorm;
        if (st) st->x0_rel_residual = r0 / bnorm;
        if (tail->nonfinite || !(r0 < bnorm)) {
            if (st) st->used_fallback = 1;
            hipLaunchKernelGGL(k_fill0, dim3(nbv), dim3(256), 0, s, n, w.u);
            PG_TRY(residual());
            PG_TRY(read_tail());
        }
        rnorm = tail->rnorm;
    }
    // The cycle state (V0, g) is in place; set the tolerance and clear flags.
    hipLaunchKernelGGL(k_set_tol, dim3(1), dim3(1), 0, s, w.ctl, tol_abs);

    const bool use_graph = o.use_graph && !prof.on;
    if (use_graph && w.graph == nullptr) {
        // Capture on a private stream (the legacy default stream cannot be
        // captured); the graph is then launched on the caller's stream.
        if (!w.graph_stream) PG_HIP(hipStreamCreateWithFlags(&w.graph_stream, hipStreamNonBlocking));
        hipGraph_t g;
        hipStream_t caller = s;
        s = w.graph_stream;
        PG_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        int rc = cycle();
        hipError_t ce = hipStreamEndCapture(s, &g);
        s = caller;
        if (rc != PETGEM_OK) return rc;
        if (ce != hipSuccess) {
            set_error(std::string("graph capture: ") + hipGetErrorString(ce));
            return PETGEM_HIP_ERROR;
        }
        hipError_t ie = hipGraphInstantiate(&w.graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) {
            set_error(std::string("graph instantiate: ") + hipGetErrorString(ie));
            return PETGEM_HIP_ERROR;
        }
    }

    int iters = 0, cycles = 0;
    int status = PETGEM_OK;
    while (true) {
        if (rnorm <= tol_abs) break;
        if (iters >= o.max_iter) { status = PETGEM_NOT_CONVERGED; break; }
        if (use_graph) {
            PG_HIP(hipGraphLaunch(w.graph, s));
        } else {
            PG_TRY(cycle());
        }
        PG_TRY(read_tail());
        iters += tail->last_m;
        ++cycles;
        rnorm = tail->rnorm;
        if (o.verbose && cycles % 10 == 0) {
            fprintf(stderr, "[petgem] GMRES cycle %d: %d iterations, true residual %.3e, %.0f ms\n", cycles,
                    iters, rnorm / bnorm, t_all.ms());
            fflush(stderr);
        }
        if (tail->nonfinite) { status = PETGEM_NONFINITE; break; }
        if (tail->last_m == 0) { status = PETGEM_NOT_CONVERGED; break; }   // stagnation
    }
    // x = D^{-1} u
    hipLaunchKernelGGL(k_scale_in, dim3(nbv), dim3(256), 0, s, n, sys->dinv, w.u, x_out);
    PG_HIP(hipGetLastError());
    prof.collect(st);
    if (st) {
        st->iters = iters;
        st->ir_steps = cycles;
        st->spmv_shape = sys->spmv_group;
        st->rel_residual = rnorm / bnorm;
        st->status = status;
        st->t_solve_ms = t_all.ms();
    }
    if (status == PETGEM_NOT_CONVERGED) set_error("GMRES reached max_iter before rtol");
    if (status == PETGEM_NONFINITE) set_error("non-finite value in the GMRES recurrence");
    return status;
}

}  // namespace petgem
