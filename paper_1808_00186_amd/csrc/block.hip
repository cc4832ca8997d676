// Multi-column Jacobi-preconditioned COCG in complex64 inside a complex128
// iterative-refinement loop, for many sources and frequencies on one mesh
// (petgem_solve with PETGEM_COCG) and for an uneven batch of meshes
// (petgem_solve_many). Not in the paper, which solves one source at a time
// with PETSc Krylov solvers (Sections 5.1-5.3); the discrete system is the
// same, A_c = K - i w_c mu0 M_sigma for each column c.
//
// Operator. Every column c of a block vector X[n][C] (row-major, so the
// C values gathered for one column index are contiguous) may have its own
// frequency: the SpMM reads the real K and M_sigma once per iteration for all
// columns and forms  y_c = K x_c - i (w_c mu0) M_sigma x_c.  Rows are cut into
// tiles of kTR rows; a tile belongs to one "segment" (one mesh of an uneven
// batch, the concatenated block-diagonal system of several meshes), and each
// (segment, column) pair carries its own Krylov scalars.
//
// COCG (complex symmetric A = A^T, Jacobi D = diag A, bilinear form u^T v):
//   r = b, x = 0, z = D^-1 r, p = z, rho = r^T z
//   repeat: q = A p; alpha = rho / p^T q; x += alpha p; r -= alpha q;
//           z = D^-1 r; rho' = r^T z; stop if |r| <= tol;
//           beta = rho' / rho; rho = rho'; p = z + beta p
// Per iteration: the SpMM (partials of p^T q in its epilogue), a reduction,
// the x / r / z update (partials of r^T z and |r|^2), a reduction, the p
// update. For one mesh with few partials the two reductions move into the
// prologues of the update kernels (see "reductions in the consumers"), so an
// iteration is three kernels; there the first updates r and z, the second x
// and p (both read p's row anyway), and a single column reads a precomputed
// complex64 D^-1. One column of one mesh on the pipelined sliced ELLPACK
// takes the fused step instead (see "fused single-column step"): the product
// also sums q^T D^-1 r and q^T D^-1 q, beta follows from the expanded next
// rho, and one vector kernel updates r, x and p: two kernels per iteration.
// A stagnation guard ends the inner solve of a column that stops improving.
// Not used, after trial: the single-reduction
// rearrangement of Chronopoulos and Gear, which carries A p by a recurrence,
// loses convergence in complex64 on the harder marine models; folding the p
// update into the SpMM (gathering z and p together) costs more than the pass
// it saves; completing the reductions in the last block of each kernel needs
// a device-wide cache write-back per block, which costs more than a reduction
// kernel.
// The SpMM shapes: CSR with nonzero lanes or column lanes, or a sliced
// ELLPACK copy of the operator (one row per lane, the rows of each tile
// ordered by length) for up to four columns, also in a software-pipelined
// form; the autotuner picks per operator and column count.
// Host loop: runs of 8-iteration groups as captured graphs (one graph per
// run length), the host reading the column states between runs while the
// next run is already queued.
// The dots are accumulated in double precision from complex64 data, per tile,
// and reduced per (segment, column) in a fixed order (bitwise reproducible).
// Refinement: r64 = b - A x64 in double precision, the inner solve runs on
// r64/|r64| in complex64 to its tolerance, x64 += |r64| d.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <map>
#include <tuple>

#include <hip/hip_ext.h>

#include "device.h"
#include "internal.h"

namespace petgem {

namespace {

constexpr int kTR = 256;        // rows per tile
constexpr int kCheck = 8;       // inner iterations between host checks (one graph)
static_assert(kCheck % 2 == 0, "the fused step's state slots alternate within a group");
constexpr int64_t kConsumerMax = 8192;   // partials a vector kernel's block may sum itself
constexpr int kConsumerTiles = 4;        // tiles per block of the in-consumer vector kernels
constexpr int kSnapRing = 32;            // host snapshot slots of the fused step (a power of two)
constexpr int kStepTiles = 8;   // tiles per block of the fused single-column step (2, 4, 16: 12, 2.5, 3.5 % slower)
constexpr int kMaxGroups = 6;   // iteration groups between two host checks (4, 8: 0.5, 1.5 % slower on a 434k-DOF mesh)

__device__ __forceinline__ float2 f2(float x, float y) { return make_float2(x, y); }

template <typename T> struct V2;
template <> struct V2<float> { using t = float2; };
template <> struct V2<double> { using t = double2; };

struct ColState {
    double2 rho, alpha, beta;
    double rn2;        // inner |r|^2 (relative to the normalised start)
    double rn2_0;      // |r|^2 at the start of the inner solve the tolerance is relative to (1, or the
                       // split residual's of an Eisenstat solve)
    double rn2_best;   // least inner |r|^2 of the current refinement step
    double scale;      // |r64| of the current refinement step
    double bnorm;      // |b|
    double rnorm64;    // true residual norm
    double tol_abs;    // rtol |b|
    double inner_tol2; // squared inner tolerance of the current refinement step
    double inner_rtol; // requested inner tolerance
    int active;        // inner iteration running
    int outer;         // not yet converged in double precision
    int breakdown;
    int iters;         // inner iterations (all refinement steps)
    int kin;           // inner iterations of the current refinement step
    int stepped;       // this iteration's alpha was applied to r (set at the beta step)
    int k_best;        // inner iteration of rn2_best
    int stalled;       // inner steps ended by the stagnation guard (all refinement steps)
    // symmetric QMR (sqmr): the quasi-minimal-residual smoothing of the iterate
    double tau2;       // tau^2, the smoothed residual's estimate (same norm as rn2)
    double cq;         // c^2 of the latest beta step: x_Q = (1 - c^2) x_Q + c^2 x
    double tmark;      // tau^2 at the last halving of tau (the plateau rule)
    int sqmr;          // this solve is SQMR
};

// Stagnation guard of the inner COCG, which has no minimisation property: a
// column whose inner |r|^2 has not improved on its best of this refinement
// step for twice the iterations the best took plus kStallIters stops its
// inner solve; the refinement step applies its correction and the next step
// restarts from the true residual. Without it one column of a 32-source block
// on the 6.9M-DOF marine mesh, after a last-bit change of its starting scale,
// wandered at inner |r| ~ 1 for 18,000 iterations instead of converging.
// (A guard that also stopped a column on a 1000-fold rise of |r|, with 500
// instead of 3000 iterations, fired on ordinary spikes of converging columns:
// their corrections raised the true residual 50-fold and the block needed
// 4-6 refinement steps instead of 3.)
constexpr int kStallIters = 3000;
__device__ __forceinline__ bool stalled_now(ColState& S, double r2) {
    if (r2 < S.rn2_best) {
        S.rn2_best = r2;
        S.k_best = S.kin;
        return false;
    }
    return S.kin - S.k_best > 2 * S.k_best + kStallIters;
}

// The last refinement step of a column solves its correction only as far as
// the target needs, with a factor 0.3 to spare (res_step). A column whose
// inner |r| hovers just above that target without a new best for half the
// iterations its best took (at least kRelaxIters) gives the margin up: it
// stops once |r| is within the target without the factor. (With a quarter,
// columns that were still converging gave the margin up, missed rtol and
// needed a fourth refinement step.) (On the
// 6.9M-unknown survey one 0.25 Hz column reached 1.04 times its target of
// 2.2e-2 at iteration 576 of its third step, then wandered for 4,000
// iterations until the guard above stopped it.)
constexpr int kRelaxIters = 100;
// In any refinement step, a column whose |r| has had no new best for as many
// iterations as its best took (at least kPlateauIters) stops at the first
// iterate whose |r| is at most 0.1 of the step's start: its correction
// still reduces the true residual tenfold, and the next refinement step
// restarts from it. (The same 0.25 Hz survey had a column reach 1.4 times the
// inner target 3e-5 at iteration 365 of its first step and wander between
// 2e-4 and 7e-3 until the guard stopped it at 4,096.) A plateau as long as
// the whole descent before it does not occur in a column that still
// converges.
constexpr int kPlateauIters = 200;
__device__ __forceinline__ bool plateau_now(const ColState& S, double r2) {
    const bool last_step = S.inner_tol2 > S.inner_rtol * S.inner_rtol;   // that one has its own rule
    return !last_step && S.kin - S.k_best >= max(kPlateauIters, S.k_best) && r2 <= 0.01 * S.rn2_0;
}
__device__ __forceinline__ bool relaxed_now(const ColState& S, double r2) {
    const bool last_step = S.inner_tol2 > S.inner_rtol * S.inner_rtol;
    return last_step && r2 <= S.inner_tol2 * S.rn2_0 / (0.3 * 0.3) &&
           S.kin - S.k_best >= max(kRelaxIters, S.k_best / 2);
}

// Operator view shared by the kernels.
struct Op {
    int n;                 // rows including padding (multiple of kTR)
    int C;                 // columns
    int ntiles, nseg;
    const int* tile_seg;   // [ntiles] or null (one segment)
    const int* seg_tile;   // [nseg+1] first tile of each segment
    const int32_t* rp;
    const int32_t* col;
    const float* K32;
    const float* M32;
    const double* K64;
    const double* M64;
    const double* Kd;      // [n]
    const double* Md;      // [n]
    const double* wmu;     // [nseg][C] w mu0
    int nrow_valid;        // rows with a matrix row (rp[i] defined for i < nrow_valid)
    // sliced-ELLPACK copy of the complex64 operator (null when absent); its
    // 64-row slices tile the kTR-row tiles exactly, with the rows of a tile
    // reordered by length (srow: the matrix row of each slice lane)
    const int32_t* sp;
    const int32_t* sw;
    const int32_t* srow;
    const int32_t* scol;
    const float* sK;
    const float* sM;
    // inner-loop launches over a subset of the tiles (an uneven batch whose
    // converged meshes drop out): block b takes tile tmap[b]; null = all
    const int* tmap;
    int nlaunch;           // tiles launched (ntiles when tmap is null)
};

__device__ __forceinline__ int tile_of(const Op& op, int b) { return op.tmap ? op.tmap[b] : b; }

// ------------------------------------------------------------ reductions
enum RedMode { RED_INIT = 0, RED_ALPHA = 1, RED_BETA = 2, RED_RES = 3, RED_X0 = 4, RED_INIT_REL = 5 };

__device__ __forceinline__ bool cfinite(double2 a) { return isfinite(a.x) && isfinite(a.y); }
__device__ __forceinline__ bool czero(double2 a) { return a.x == 0.0 && a.y == 0.0; }

// alpha = rho / p^T q (or breakdown) for an active column
__device__ __forceinline__ void step_alpha(ColState& S, double2 pq) {
    if (!cfinite(pq) || czero(pq)) {
        S.active = 0;
        S.breakdown = 1;
        S.alpha = make_double2(0.0, 0.0);
    } else {
        S.alpha = cdiv(S.rho, pq);
    }
}

// convergence test on |r|^2 and beta = rho' / rho for an active column
// (counting the update that produced r)
// The scalar step of SQMR (Section 5.3 names SQMR with SOR as the paper's
// single-process solver). Its recurrence is COCG's (rho, beta as in
// step_beta); the quasi-minimal-residual smoothing of the iterate takes, from
// the new residual norm |r|^2 = r2, theta^2 = r2 / tau^2, c^2 = 1 / (1 +
// theta^2) and tau^2 <- tau^2 theta^2 c^2, and the smoothed iterate is
// x_Q = (1 - c^2) x_Q + c^2 x (written by the update kernels). tau falls
// monotonically, so the inner solve stops once tau is within the target, or
// once tau has not halved for as many iterations as its last halving took
// (at least kPlateauIters). tau bounds the smoothed residual only when the
// residuals are orthogonal; COCG's are orthogonal in the bilinear form, not
// in the Euclidean one, and where the unsmoothed residual diverges tau still
// falls while the smoothed residual does not (a refinement step then gains
// nothing).
__device__ __forceinline__ void sqmr_beta(ColState& S, double2 rz, double r2) {
    S.iters += 1;
    S.kin += 1;
    S.rn2 = r2;
    if (!isfinite(r2) || !cfinite(rz)) {
        S.active = 0;
        S.breakdown = 1;
        return;
    }
    const double th2 = S.tau2 > 0.0 ? r2 / S.tau2 : 0.0;
    const double c2 = 1.0 / (1.0 + th2);
    S.tau2 = S.tau2 * th2 * c2;
    S.cq = c2;
    S.rn2_best = S.tau2;
    if (S.tau2 <= S.inner_tol2 * S.rn2_0) {
        S.active = 0;
        return;
    }
    if (S.tau2 <= 0.25 * S.tmark) {
        S.tmark = S.tau2;
        S.k_best = S.kin;
    } else if (S.kin - S.k_best >= max(kPlateauIters, S.k_best)) {
        S.active = 0;
        S.stalled += 1;
        return;
    }
    if (czero(S.rho)) {
        S.active = 0;
        S.breakdown = 1;
        return;
    }
    S.beta = cdiv(rz, S.rho);
    S.rho = rz;
}

__device__ __forceinline__ void step_beta(ColState& S, double2 rz, double r2) {
    S.iters += 1;
    S.kin += 1;
    S.rn2 = r2;
    if (!isfinite(r2) || !cfinite(rz)) {
        S.active = 0;
        S.breakdown = 1;
    } else if (r2 <= S.inner_tol2 * S.rn2_0) {
        S.active = 0;
    } else if (stalled_now(S, r2)) {
        S.active = 0;
        S.stalled += 1;
    } else if (relaxed_now(S, r2)) {
        S.active = 0;
    } else if (plateau_now(S, r2)) {
        S.active = 0;
        S.stalled += 1;
    } else if (czero(S.rho)) {
        S.active = 0;
        S.breakdown = 1;
    } else {
        S.beta = cdiv(rz, S.rho);
        S.rho = rz;
    }
}

// The true residual norm rn of the current iterate is known: the outer
// convergence test and the next refinement step's inner tolerance.
__device__ __forceinline__ void res_step(ColState& S, double rn, int first) {
    S.rnorm64 = rn;
    if (first) S.bnorm = rn;
    S.scale = rn;
    S.outer = S.outer && !(rn <= S.tol_abs) && isfinite(rn);
    // no need to solve the correction more accurately than the target asks:
    // a factor 0.3 below rtol |b| / |r64| leaves a safety margin
    const double need = rn > 0.0 ? 0.3 * S.tol_abs / rn : 1.0;
    const double it = fmax(S.inner_rtol, fmin(need, 0.5));
    S.inner_tol2 = it * it;
}

// The scalar step of one (segment, column) once its sums a, b are known.
__device__ void apply_red(ColState& S, int mode, int first, double2 a, double2 b) {
    if (mode == RED_INIT || mode == RED_INIT_REL) {   // a = r^T z, b.x = |r|^2 of the start
        S.rho = a;
        S.rn2 = b.x;
        S.rn2_0 = mode == RED_INIT_REL ? b.x : 1.0;   // else normalised: |r| = 1
        S.rn2_best = b.x;
        S.k_best = 0;
        S.kin = 0;
        S.beta = make_double2(0.0, 0.0);
        S.active = S.outer && cfinite(a) && !czero(a);
        S.breakdown = 0;
        S.stepped = 0;
        S.tau2 = b.x;                  // tau_0 = |r_0| (x_Q = x = 0)
        S.tmark = b.x;
        S.cq = 0.0;
    } else if (mode == RED_ALPHA) {    // a = p^T q
        step_alpha(S, a);
    } else if (mode == RED_BETA) {     // a = r^T z (new), b.x = |r|^2
        S.stepped = 1;
        if (S.sqmr) sqmr_beta(S, a, b.x);
        else step_beta(S, a, b.x);
    } else if (mode == RED_X0) {       // a = w^H b, b.x = |w|^2 for w = A x0
        // a zero right-hand side (its residual never formed) has x = 0; a guess
        // that already meets the tolerance is scaled all the same
        S.alpha = (S.bnorm > 0.0 && b.x > 0.0 && isfinite(b.x) && cfinite(a)) ? cscale(a, 1.0 / b.x)
                                                                             : make_double2(0.0, 0.0);
    } else {                           // RED_RES: a.x = |b - A x|^2
        res_step(S, sqrt(a.x), first);
    }
}

__device__ __forceinline__ bool red_skips(const ColState& S, int mode, int first) {
    return ((mode == RED_ALPHA || mode == RED_BETA) && !S.active) || (mode == RED_RES && !first && !S.outer);
}

// One block per (segment, column): fixed-order sums over the segment's tiles
// (pp0 / pp1 partial slots per tile), then the scalar step of that column.
__global__ void __launch_bounds__(1024)
k_reduce(Op op, const double2* __restrict__ p0, int pp0, const double2* __restrict__ p1, int pp1,
         ColState* __restrict__ st, int mode, int first) {
    __shared__ double2 sa[1024], sb[1024];
    const int sc = blockIdx.x;
    const int s = sc / op.C, c = sc % op.C;
    ColState& S = st[sc];
    if (red_skips(S, mode, first)) {
        if (mode == RED_BETA && threadIdx.x == 0) S.stepped = 0;   // inactive: no alpha was applied
        return;
    }
    const int t0 = op.seg_tile[s], t1 = op.seg_tile[s + 1];
    double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
    {
        const int e0 = t0 * pp0, e1 = t1 * pp0;
        for (int e = e0 + threadIdx.x; e < e1; e += 1024 * 8) {
            double2 v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int k = e + 1024 * u;
                v[u] = k < e1 ? p0[(size_t)k * op.C + c] : make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) a = cadd(a, v[u]);
        }
    }
    if (p1) {
        const int e0 = t0 * pp1, e1 = t1 * pp1;
        for (int e = e0 + threadIdx.x; e < e1; e += 1024 * 8) {
            double2 v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int k = e + 1024 * u;
                v[u] = k < e1 ? p1[(size_t)k * op.C + c] : make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) b = cadd(b, v[u]);
        }
    }
    // fixed-shape tree: shuffles inside each wave, then the 16 wave sums
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    a.x = wave_sum(a.x); a.y = wave_sum(a.y);
    b.x = wave_sum(b.x); b.y = wave_sum(b.y);
    if (lane == 0) { sa[wave] = a; sb[wave] = b; }
    __syncthreads();
    if (threadIdx.x != 0) return;
    a = sa[0];
    b = sb[0];
    for (int k = 1; k < 16; ++k) { a = cadd(a, sa[k]); b = cadd(b, sb[k]); }
    apply_red(S, mode, first, a, b);
}

// One block per column of one system, on partials stored column by column
// (column c's n0 slots from p0 + c * s0, likewise p1): fixed-order sums, then
// the scalar step of that column. A block reads only its own column's slots,
// contiguously; k_reduce's row-major slots would cost it a cache line per
// 16-byte partial.
__global__ void __launch_bounds__(1024)
k_reduce_cm(const double2* __restrict__ p0, int n0, int64_t s0, const double2* __restrict__ p1, int n1, int64_t s1,
            ColState* __restrict__ st, int mode) {
    __shared__ double2 sa[16], sb[16];
    const int c = blockIdx.x;
    ColState& S = st[c];
    if (red_skips(S, mode, 0)) {
        if (mode == RED_BETA && threadIdx.x == 0) S.stepped = 0;   // inactive: no alpha was applied
        return;
    }
    double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
    {
        const double2* q = p0 + (size_t)c * s0;
        for (int e = threadIdx.x; e < n0; e += 1024 * 8) {
            double2 v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int k = e + 1024 * u;
                v[u] = k < n0 ? q[k] : make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) a = cadd(a, v[u]);
        }
    }
    if (p1) {
        const double2* q = p1 + (size_t)c * s1;
        for (int e = threadIdx.x; e < n1; e += 1024 * 8) {
            double2 v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int k = e + 1024 * u;
                v[u] = k < n1 ? q[k] : make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) b = cadd(b, v[u]);
        }
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    a.x = wave_sum(a.x); a.y = wave_sum(a.y);
    b.x = wave_sum(b.x); b.y = wave_sum(b.y);
    if (lane == 0) { sa[wave] = a; sb[wave] = b; }
    __syncthreads();
    if (threadIdx.x != 0) return;
    a = sa[0];
    b = sb[0];
    for (int k = 1; k < 16; ++k) { a = cadd(a, sa[k]); b = cadd(b, sb[k]); }
    apply_red(S, mode, 0, a, b);
}

// ------------------------------------------------------------------ SpMM
// EPI 2: Y = B - A X in the template type and partial[..][c].x = sum_i |Y_ic|^2.
// EPI 1: Y = A X and partial[..][c] = sum_i X_ic Y_ic (unconjugated).
// Column-lane variant: LPR lanes per row, CPL consecutive columns per lane.
// Columns whose Krylov solve has finished (EPI 1: inner `active` clear; EPI 2:
// refinement `outer` clear) are skipped: no gathers, no writes, zero partials.
__device__ __forceinline__ bool col_live(const ColState* st, int sc, int EPI_) {
    return EPI_ == 2 ? st[sc].outer != 0 : st[sc].active != 0;
}

template <typename T, int LPR, int CPL, int EPI>
__global__ void __launch_bounds__(256)
k_spmm_c(Op op, const ColState* __restrict__ st, const typename V2<T>::t* __restrict__ X,
         const typename V2<T>::t* __restrict__ B, typename V2<T>::t* __restrict__ Y,
         double2* __restrict__ partial) {
    using T2 = typename V2<T>::t;
    const T* __restrict__ Kv = nullptr;
    const T* __restrict__ Mv = nullptr;
    if constexpr (sizeof(T) == 4) { Kv = op.K32; Mv = op.M32; } else { Kv = op.K64; Mv = op.M64; }
    constexpr int RPB = 256 / LPR;
    __shared__ double2 red[RPB][LPR * CPL];
    const int tile = tile_of(op, xcd_block(blockIdx.x, gridDim.x));
    const int slot = threadIdx.x / LPR, l = threadIdx.x % LPR;
    const int C = op.C;
    const int seg = op.tile_seg ? op.tile_seg[tile] : 0;
    T wmu[CPL];
    bool live[CPL];
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
        const int c = l * CPL + u;
        live[u] = c < C && col_live(st, seg * C + c, EPI);
        wmu[u] = c < C ? (T)op.wmu[seg * C + c] : (T)0;
    }
    double2 pacc[CPL];
#pragma unroll
    for (int u = 0; u < CPL; ++u) pacc[u] = make_double2(0.0, 0.0);
    for (int r0 = 0; r0 < kTR; r0 += RPB) {
        const int i = tile * kTR + r0 + slot;
        if (i >= op.nrow_valid) continue;
        T2 ak[CPL], am[CPL];
#pragma unroll
        for (int u = 0; u < CPL; ++u) { ak[u].x = ak[u].y = (T)0; am[u].x = am[u].y = (T)0; }
        const int32_t e = op.rp[i + 1];
        // 4 nonzeros in flight: indices and values first, then the gathers
        for (int32_t k0 = op.rp[i]; k0 < e; k0 += 4) {
            int32_t cj[4];
            T kv[4], mv[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const bool ok = k0 + q < e;
                cj[q] = ok ? op.col[k0 + q] : -1;
                kv[q] = ok ? Kv[k0 + q] : (T)0;
                mv[q] = ok ? Mv[k0 + q] : (T)0;
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (cj[q] < 0) continue;
                const T2* xr = X + (size_t)cj[q] * C + l * CPL;
#pragma unroll
                for (int u = 0; u < CPL; ++u) {
                    if (live[u]) {
                        const T2 xv = xr[u];
                        ak[u].x += kv[q] * xv.x; ak[u].y += kv[q] * xv.y;
                        am[u].x += mv[q] * xv.x; am[u].y += mv[q] * xv.y;
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < CPL; ++u) {
            const int c = l * CPL + u;
            if (!live[u]) continue;
            T2 y;
            y.x = ak[u].x + wmu[u] * am[u].y;   // K x - i wmu M x
            y.y = ak[u].y - wmu[u] * am[u].x;
            const size_t o = (size_t)i * C + c;
            if constexpr (EPI == 2) {
                const T2 bb = B[o];
                y.x = bb.x - y.x;
                y.y = bb.y - y.y;
                pacc[u].x += (double)y.x * (double)y.x + (double)y.y * (double)y.y;
            } else {
                const T2 xo = X[o];
                pacc[u].x += (double)xo.x * (double)y.x - (double)xo.y * (double)y.y;
                pacc[u].y += (double)xo.x * (double)y.y + (double)xo.y * (double)y.x;
            }
            Y[o] = y;
        }
    }
#pragma unroll
    for (int u = 0; u < CPL; ++u) red[slot][l * CPL + u] = pacc[u];
    for (int w = RPB >> 1; w > 0; w >>= 1) {
        __syncthreads();
        if (slot < w)
#pragma unroll
            for (int u = 0; u < CPL; ++u)
                red[slot][l * CPL + u] = cadd(red[slot][l * CPL + u], red[slot + w][l * CPL + u]);
    }
    __syncthreads();
    for (int c = threadIdx.x; c < C && c < LPR * CPL; c += 256) partial[(size_t)tile * C + c] = red[0][c];
}

// Column-lane variant with the row's nonzeros spread over its lanes ("kind
// 6"): the LPR lanes of a row load NB consecutive (column, K, M) entries with
// coalesced accesses (lane l takes entries l, l + LPR, ...), then every lane
// takes the whole chunk's indices and values from its neighbours by shuffles
// within the row's lane group and issues all NB gathers of its CPL columns
// before the first accumulation. A row of up to NB nonzeros costs one
// dependent round trip (the entries, then the gathers) instead of one per four
// nonzeros; the sums keep the row's nonzero order. Rows of a wave with
// different lengths take different trip counts; a row's lane group is always
// active or inactive as a whole, so the shuffles read active lanes only.
template <typename T, int LPR, int CPL, int NB, int EPI>
__global__ void __launch_bounds__(256)
k_spmm_g(Op op, const ColState* __restrict__ st, const typename V2<T>::t* __restrict__ X,
         const typename V2<T>::t* __restrict__ B, typename V2<T>::t* __restrict__ Y,
         double2* __restrict__ partial) {
    using T2 = typename V2<T>::t;
    static_assert(LPR <= kWave && (LPR & (LPR - 1)) == 0, "a row's lanes are a power-of-two group of one wave");
    constexpr int NH = (NB + LPR - 1) / LPR;   // entry loads per lane and trip
    const T* __restrict__ Kv = nullptr;
    const T* __restrict__ Mv = nullptr;
    if constexpr (sizeof(T) == 4) { Kv = op.K32; Mv = op.M32; } else { Kv = op.K64; Mv = op.M64; }
    constexpr int RPB = 256 / LPR;
    __shared__ double2 red[RPB][LPR * CPL];
    const int tile = tile_of(op, xcd_block(blockIdx.x, gridDim.x));
    const int slot = threadIdx.x / LPR, l = threadIdx.x % LPR;
    const int C = op.C;
    const int seg = op.tile_seg ? op.tile_seg[tile] : 0;
    T wmu[CPL];
    bool live[CPL];
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
        const int c = l * CPL + u;
        live[u] = c < C && col_live(st, seg * C + c, EPI);
        wmu[u] = c < C ? (T)op.wmu[seg * C + c] : (T)0;
    }
    double2 pacc[CPL];
#pragma unroll
    for (int u = 0; u < CPL; ++u) pacc[u] = make_double2(0.0, 0.0);
    for (int r0 = 0; r0 < kTR; r0 += RPB) {
        const int i = tile * kTR + r0 + slot;
        const bool okrow = i < op.nrow_valid;
        int32_t kb = okrow ? op.rp[i] : 0;
        const int32_t ke = okrow ? op.rp[i + 1] : 0;
        T2 ak[CPL], am[CPL];
#pragma unroll
        for (int u = 0; u < CPL; ++u) { ak[u].x = ak[u].y = (T)0; am[u].x = am[u].y = (T)0; }
        for (; kb < ke; kb += NB) {
            int32_t cj[NH];
            T kv[NH], mv[NH];
#pragma unroll
            for (int h = 0; h < NH; ++h) {
                const int32_t k = kb + h * LPR + l;
                const bool ok = h * LPR + l < NB && k < ke;
                cj[h] = ok ? op.col[k] : 0;
                kv[h] = ok ? Kv[k] : (T)0;
                mv[h] = ok ? Mv[k] : (T)0;
            }
            T2 xv[NB][CPL];
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                const int c = __shfl(cj[q / LPR], q % LPR, LPR);
                const bool ok = kb + q < ke;
                const T2* xr = X + (size_t)c * C + l * CPL;
#pragma unroll
                for (int u = 0; u < CPL; ++u) {
                    if (ok && live[u]) xv[q][u] = xr[u];
                    else { xv[q][u].x = (T)0; xv[q][u].y = (T)0; }
                }
            }
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                const T kq = __shfl(kv[q / LPR], q % LPR, LPR);
                const T mq = __shfl(mv[q / LPR], q % LPR, LPR);
#pragma unroll
                for (int u = 0; u < CPL; ++u) {
                    ak[u].x += kq * xv[q][u].x; ak[u].y += kq * xv[q][u].y;
                    am[u].x += mq * xv[q][u].x; am[u].y += mq * xv[q][u].y;
                }
            }
        }
        if (!okrow) continue;
#pragma unroll
        for (int u = 0; u < CPL; ++u) {
            const int c = l * CPL + u;
            if (!live[u]) continue;
            T2 y;
            y.x = ak[u].x + wmu[u] * am[u].y;   // K x - i wmu M x
            y.y = ak[u].y - wmu[u] * am[u].x;
            const size_t o = (size_t)i * C + c;
            if constexpr (EPI == 2) {
                const T2 bb = B[o];
                y.x = bb.x - y.x;
                y.y = bb.y - y.y;
                pacc[u].x += (double)y.x * (double)y.x + (double)y.y * (double)y.y;
            } else {
                const T2 xo = X[o];
                pacc[u].x += (double)xo.x * (double)y.x - (double)xo.y * (double)y.y;
                pacc[u].y += (double)xo.x * (double)y.y + (double)xo.y * (double)y.x;
            }
            Y[o] = y;
        }
    }
#pragma unroll
    for (int u = 0; u < CPL; ++u) red[slot][l * CPL + u] = pacc[u];
    for (int w = RPB >> 1; w > 0; w >>= 1) {
        __syncthreads();
        if (slot < w)
#pragma unroll
            for (int u = 0; u < CPL; ++u)
                red[slot][l * CPL + u] = cadd(red[slot][l * CPL + u], red[slot + w][l * CPL + u]);
    }
    __syncthreads();
    for (int c = threadIdx.x; c < C && c < LPR * CPL; c += 256) partial[(size_t)tile * C + c] = red[0][c];
}

// Nonzero-lane variant for few columns: G lanes share the nonzeros of a row,
// each lane accumulates all (<= CM) columns, then a shuffle reduction.
template <typename T, int G, int CM, int EPI>
__global__ void __launch_bounds__(256)
k_spmm_n(Op op, const ColState* __restrict__ st, const typename V2<T>::t* __restrict__ X,
         const typename V2<T>::t* __restrict__ B, typename V2<T>::t* __restrict__ Y,
         double2* __restrict__ partial) {
    using T2 = typename V2<T>::t;
    const T* __restrict__ Kv = nullptr;
    const T* __restrict__ Mv = nullptr;
    if constexpr (sizeof(T) == 4) { Kv = op.K32; Mv = op.M32; } else { Kv = op.K64; Mv = op.M64; }
    constexpr int RPB = 256 / G;      // rows per block: kTR / RPB = G blocks per tile
    __shared__ double2 red[4][CM];
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    const int tile = tile_of(op, lb / G), pass = lb % G;
    const int bid = tile * G + pass;   // partial slot
    const int slot = threadIdx.x / G, l = threadIdx.x % G;
    const int C = op.C;
    const int seg = op.tile_seg ? op.tile_seg[tile] : 0;
    double2 pacc[CM];
    bool live[CM], any = false;
#pragma unroll
    for (int u = 0; u < CM; ++u) {
        pacc[u] = make_double2(0.0, 0.0);
        live[u] = u < C && col_live(st, seg * C + u, EPI);
        any = any || live[u];
    }
    // every column of this segment stopped: nothing reads this tile's partials
    if (!any) return;
    {
        const int i = tile * kTR + pass * RPB + slot;
        if (any && i < op.nrow_valid) {   // the whole G-lane group shares i and seg
        T2 ak[CM], am[CM];
#pragma unroll
        for (int u = 0; u < CM; ++u) { ak[u].x = ak[u].y = (T)0; am[u].x = am[u].y = (T)0; }
        const int32_t e = op.rp[i + 1];
        // 4 nonzeros per lane in flight: all index and value loads first
        for (int32_t k0 = op.rp[i] + l; k0 < e; k0 += 4 * G) {
            int32_t cj[4];
            T kv[4], mv[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int32_t k = k0 + q * G;
                const bool ok = k < e;
                cj[q] = ok ? op.col[k] : -1;
                kv[q] = ok ? Kv[k] : (T)0;
                mv[q] = ok ? Mv[k] : (T)0;
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (cj[q] < 0) continue;
                const T2* xr = X + (size_t)cj[q] * C;
#pragma unroll
                for (int u = 0; u < CM; ++u) {
                    if (live[u]) {
                        const T2 xv = xr[u];
                        ak[u].x += kv[q] * xv.x; ak[u].y += kv[q] * xv.y;
                        am[u].x += mv[q] * xv.x; am[u].y += mv[q] * xv.y;
                    }
                }
            }
        }
#pragma unroll
        for (int off = G / 2; off > 0; off >>= 1) {
#pragma unroll
            for (int u = 0; u < CM; ++u) {
                ak[u].x += __shfl_xor(ak[u].x, off, G); ak[u].y += __shfl_xor(ak[u].y, off, G);
                am[u].x += __shfl_xor(am[u].x, off, G); am[u].y += __shfl_xor(am[u].y, off, G);
            }
        }
        if (l == 0) {
#pragma unroll
            for (int u = 0; u < CM; ++u) {
                if (!live[u]) continue;
                const T w = (T)op.wmu[seg * C + u];
                T2 y;
                y.x = ak[u].x + w * am[u].y;
                y.y = ak[u].y - w * am[u].x;
                const size_t o = (size_t)i * C + u;
                if constexpr (EPI == 2) {
                    const T2 bb = B[o];
                    y.x = bb.x - y.x;
                    y.y = bb.y - y.y;
                    pacc[u].x += (double)y.x * (double)y.x + (double)y.y * (double)y.y;
                } else {
                    const T2 xo = X[o];
                    pacc[u].x += (double)xo.x * (double)y.x - (double)xo.y * (double)y.y;
                    pacc[u].y += (double)xo.x * (double)y.y + (double)xo.y * (double)y.x;
                }
                Y[o] = y;
            }
        }
        }
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int u = 0; u < CM; ++u) {
        const double sx = wave_sum(pacc[u].x), sy = wave_sum(pacc[u].y);
        if (lane == 0) red[wave][u] = make_double2(sx, sy);
    }
    __syncthreads();
    if ((int)threadIdx.x < C && (int)threadIdx.x < CM) {
        const int u = threadIdx.x;
        double2 s = red[0][u];
        s = cadd(s, red[1][u]);
        s = cadd(s, red[2][u]);
        s = cadd(s, red[3][u]);
        partial[(size_t)bid * C + u] = s;
    }
}

// Sliced-ELLPACK variant (EPI 1, complex64, C <= CM <= 4): one row per lane,
// the block's four wavefronts take the four 64-row slices of one tile; U
// slice columns (index and values) are loaded ahead of their gathers.
template <int CM, int U>
__global__ void __launch_bounds__(256)
k_spmm_s(Op op, const ColState* __restrict__ st, const float2* __restrict__ X, float2* __restrict__ Y,
         double2* __restrict__ partial) {
    __shared__ double2 red[4][CM];
    const int tile = tile_of(op, xcd_block(blockIdx.x, gridDim.x));
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int sl = tile * 4 + wave;
    const int i = op.srow[sl * 64 + lane];
    const int C = op.C;
    const int seg = op.tile_seg ? op.tile_seg[tile] : 0;
    double2 pacc[CM];
    float wmu[CM];
    bool live[CM], any = false;
#pragma unroll
    for (int u = 0; u < CM; ++u) {
        pacc[u] = make_double2(0.0, 0.0);
        live[u] = u < C && col_live(st, seg * C + u, 1);
        any = any || live[u];
        wmu[u] = u < C ? (float)op.wmu[seg * C + u] : 0.f;
    }
    // every column of this segment stopped: nothing reads this tile's partials
    if (!any) return;
    if (any) {   // the same for the whole block (one segment)
        float2 ak[CM], am[CM];
#pragma unroll
        for (int u = 0; u < CM; ++u) { ak[u] = f2(0.f, 0.f); am[u] = f2(0.f, 0.f); }
        const int base = op.sp[sl], wd = op.sw[sl];
        int k = 0;
        for (; k + U <= wd; k += U) {
            int32_t cj[U];
            float kv[U], mv[U];
#pragma unroll
            for (int q = 0; q < U; ++q) {
                const int e = base + (k + q) * 64 + lane;
                cj[q] = op.scol[e];
                kv[q] = op.sK[e];
                mv[q] = op.sM[e];
            }
#pragma unroll
            for (int q = 0; q < U; ++q) {
                const float2* xr = X + (size_t)cj[q] * C;
#pragma unroll
                for (int u = 0; u < CM; ++u) {
                    if (live[u]) {
                        const float2 xv = xr[u];
                        ak[u].x += kv[q] * xv.x; ak[u].y += kv[q] * xv.y;
                        am[u].x += mv[q] * xv.x; am[u].y += mv[q] * xv.y;
                    }
                }
            }
        }
        for (; k < wd; ++k) {
            const int e = base + k * 64 + lane;
            const float kv = op.sK[e], mv = op.sM[e];
            const float2* xr = X + (size_t)op.scol[e] * C;
#pragma unroll
            for (int u = 0; u < CM; ++u) {
                if (live[u]) {
                    const float2 xv = xr[u];
                    ak[u].x += kv * xv.x; ak[u].y += kv * xv.y;
                    am[u].x += mv * xv.x; am[u].y += mv * xv.y;
                }
            }
        }
        if (i < op.nrow_valid) {
#pragma unroll
            for (int u = 0; u < CM; ++u) {
                if (!live[u]) continue;
                float2 y;
                y.x = ak[u].x + wmu[u] * am[u].y;   // K x - i wmu M x
                y.y = ak[u].y - wmu[u] * am[u].x;
                const size_t o = (size_t)i * C + u;
                const float2 xo = X[o];
                pacc[u].x += (double)xo.x * (double)y.x - (double)xo.y * (double)y.y;
                pacc[u].y += (double)xo.x * (double)y.y + (double)xo.y * (double)y.x;
                Y[o] = y;
            }
        }
    }
#pragma unroll
    for (int u = 0; u < CM; ++u) {
        const double sx = wave_sum(pacc[u].x), sy = wave_sum(pacc[u].y);
        if (lane == 0) red[wave][u] = make_double2(sx, sy);
    }
    __syncthreads();
    if ((int)threadIdx.x < C && (int)threadIdx.x < CM) {
        const int u = threadIdx.x;
        partial[(size_t)tile * C + u] = cadd(cadd(red[0][u], red[1][u]), cadd(red[2][u], red[3][u]));
    }
}

// Software-pipelined sliced-ELLPACK variant: the same layout and epilogue
// as k_spmm_s, but the indices and values of the next U slice columns are
// loaded before the gathers of the current U, so their latency overlaps.
template <int CM, int U>
__global__ void __launch_bounds__(256)
k_spmm_sp(Op op, const ColState* __restrict__ st, const float2* __restrict__ X, float2* __restrict__ Y,
         double2* __restrict__ partial) {
    __shared__ double2 red[4][CM];
    const int tile = tile_of(op, xcd_block(blockIdx.x, gridDim.x));
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int sl = tile * 4 + wave;
    const int i = op.srow[sl * 64 + lane];
    const int C = op.C;
    const int seg = op.tile_seg ? op.tile_seg[tile] : 0;
    double2 pacc[CM];
    float wmu[CM];
    bool live[CM], any = false;
#pragma unroll
    for (int u = 0; u < CM; ++u) {
        pacc[u] = make_double2(0.0, 0.0);
        live[u] = u < C && col_live(st, seg * C + u, 1);
        any = any || live[u];
        wmu[u] = u < C ? (float)op.wmu[seg * C + u] : 0.f;
    }
    // every column of this segment stopped: nothing reads this tile's partials
    if (!any) return;
    if (any) {   // the same for the whole block (one segment)
        float2 ak[CM], am[CM];
#pragma unroll
        for (int u = 0; u < CM; ++u) { ak[u] = f2(0.f, 0.f); am[u] = f2(0.f, 0.f); }
        const int base = op.sp[sl], wd = op.sw[sl];
        // slice columns k .. k+U-1 (past the width: zero values, own row)
        int32_t cj[U];
        float kv[U], mv[U];
        auto fetch = [&](int k, int32_t* c, float* kk, float* mm) {
#pragma unroll
            for (int q = 0; q < U; ++q) {
                if (k + q < wd) {
                    const int e = base + (k + q) * 64 + lane;
                    c[q] = op.scol[e];
                    kk[q] = op.sK[e];
                    mm[q] = op.sM[e];
                } else {
                    c[q] = i < op.nrow_valid ? i : 0;
                    kk[q] = 0.f;
                    mm[q] = 0.f;
                }
            }
        };
        fetch(0, cj, kv, mv);
        for (int k = 0; k < wd; k += U) {
            float2 xv[U][CM];
#pragma unroll
            for (int q = 0; q < U; ++q) {
                const float2* xr = X + (size_t)cj[q] * C;
#pragma unroll
                for (int u = 0; u < CM; ++u) xv[q][u] = live[u] ? xr[u] : f2(0.f, 0.f);
            }
            int32_t cn[U];
            float kn[U], mn[U];
            if (k + U < wd) fetch(k + U, cn, kn, mn);
#pragma unroll
            for (int q = 0; q < U; ++q)
#pragma unroll
                for (int u = 0; u < CM; ++u) {
                    ak[u].x += kv[q] * xv[q][u].x; ak[u].y += kv[q] * xv[q][u].y;
                    am[u].x += mv[q] * xv[q][u].x; am[u].y += mv[q] * xv[q][u].y;
                }
            if (k + U < wd) {
#pragma unroll
                for (int q = 0; q < U; ++q) { cj[q] = cn[q]; kv[q] = kn[q]; mv[q] = mn[q]; }
            }
        }
        if (i < op.nrow_valid) {
#pragma unroll
            for (int u = 0; u < CM; ++u) {
                if (!live[u]) continue;
                float2 y;
                y.x = ak[u].x + wmu[u] * am[u].y;   // K x - i wmu M x
                y.y = ak[u].y - wmu[u] * am[u].x;
                const size_t o = (size_t)i * C + u;
                const float2 xo = X[o];
                pacc[u].x += (double)xo.x * (double)y.x - (double)xo.y * (double)y.y;
                pacc[u].y += (double)xo.x * (double)y.y + (double)xo.y * (double)y.x;
                Y[o] = y;
            }
        }
    }
#pragma unroll
    for (int u = 0; u < CM; ++u) {
        const double sx = wave_sum(pacc[u].x), sy = wave_sum(pacc[u].y);
        if (lane == 0) red[wave][u] = make_double2(sx, sy);
    }
    __syncthreads();
    if ((int)threadIdx.x < C && (int)threadIdx.x < CM) {
        const int u = threadIdx.x;
        partial[(size_t)tile * C + u] = cadd(cadd(red[0][u], red[1][u]), cadd(red[2][u], red[3][u]));
    }
}

__device__ __forceinline__ float2 cmulf(float2 a, float2 b) {
    return f2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Single-column form of k_spmm_sp for the fused COCG step: besides y = A x
// and p^T q it forms q^T D^-1 r and q^T D^-1 q from each row's r and D^-1
// (three partials per block, in that order, each in its own plane of
// gridDim.x values so that the step reads each plane coalesced). They give the next
// rho = (r - alpha q)^T D^-1 (r - alpha q) before r itself is updated. A
// block of W waves takes W consecutive 64-row slices (8 and 16 waves per
// block, i.e. fewer partials for the step to sum, measured no faster than 4).
template <int U, int W>
__global__ void __launch_bounds__(64 * W)
k_spmm_spb(Op op, const ColState* __restrict__ st, const float2* __restrict__ X, float2* __restrict__ Y,
           const float2* __restrict__ R, const float2* __restrict__ dinv, double2* __restrict__ partial) {
    __shared__ double2 red[W][3];
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int sl = blk * W + wave;
    const bool slice = sl < op.ntiles * 4;   // the last block may reach past the last slice
    const int i = slice ? op.srow[sl * 64 + lane] : op.n;
    if (!st[0].active) return;   // stopped: nothing reads the partials
    const float wmu = (float)op.wmu[0];
    const bool row = slice && i < op.nrow_valid;
    // this row's r and D^-1 do not depend on the product: loaded first
    const float2 rv = row ? R[i] : f2(0.f, 0.f);
    const float2 dv = row ? dinv[i] : f2(0.f, 0.f);
    float2 ak = f2(0.f, 0.f), am = f2(0.f, 0.f);
    const int base = slice ? op.sp[sl] : 0, wd = slice ? op.sw[sl] : 0;
    int32_t cj[U];
    float kv[U], mv[U];
    auto fetch = [&](int k, int32_t* c, float* kk, float* mm) {
#pragma unroll
        for (int q = 0; q < U; ++q) {
            if (k + q < wd) {
                const int e = base + (k + q) * 64 + lane;
                c[q] = op.scol[e];
                kk[q] = op.sK[e];
                mm[q] = op.sM[e];
            } else {
                c[q] = row ? i : 0;
                kk[q] = 0.f;
                mm[q] = 0.f;
            }
        }
    };
    fetch(0, cj, kv, mv);
    for (int k = 0; k < wd; k += U) {
        float2 xv[U];
#pragma unroll
        for (int q = 0; q < U; ++q) xv[q] = X[cj[q]];
        int32_t cn[U];
        float kn[U], mn[U];
        if (k + U < wd) fetch(k + U, cn, kn, mn);
#pragma unroll
        for (int q = 0; q < U; ++q) {
            ak.x += kv[q] * xv[q].x; ak.y += kv[q] * xv[q].y;
            am.x += mv[q] * xv[q].x; am.y += mv[q] * xv[q].y;
        }
        if (k + U < wd) {
#pragma unroll
            for (int q = 0; q < U; ++q) { cj[q] = cn[q]; kv[q] = kn[q]; mv[q] = mn[q]; }
        }
    }
    double2 pq = make_double2(0.0, 0.0), qzr = pq, qzq = pq;
    if (row) {
        float2 y;
        y.x = ak.x + wmu * am.y;   // K x - i wmu M x
        y.y = ak.y - wmu * am.x;
        const float2 xo = X[i];
        const float2 zr = cmulf(rv, dv), zq = cmulf(y, dv);
        pq.x = (double)xo.x * y.x - (double)xo.y * y.y;
        pq.y = (double)xo.x * y.y + (double)xo.y * y.x;
        qzr.x = (double)y.x * zr.x - (double)y.y * zr.y;
        qzr.y = (double)y.x * zr.y + (double)y.y * zr.x;
        qzq.x = (double)y.x * zq.x - (double)y.y * zq.y;
        qzq.y = (double)y.x * zq.y + (double)y.y * zq.x;
        Y[i] = y;
    }
    const double s0 = wave_sum(pq.x), s1 = wave_sum(pq.y), s2 = wave_sum(qzr.x), s3 = wave_sum(qzr.y),
                 s4 = wave_sum(qzq.x), s5 = wave_sum(qzq.y);
    if (lane == 0) {
        red[wave][0] = make_double2(s0, s1);
        red[wave][1] = make_double2(s2, s3);
        red[wave][2] = make_double2(s4, s5);
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const int u = threadIdx.x;
        double2 t = red[0][u];
#pragma unroll
        for (int k = 1; k < W; ++k) t = cadd(t, red[k][u]);
        partial[(size_t)u * gridDim.x + blk] = t;   // three planes of one partial per block
    }
}

// waves per block of the fused step's product
constexpr int kSpbWaves = 4;

// Fixed-shape sums over the row slots of a CP-lane row layout (thread t holds
// column t % CP of slot t / CP); the results for column c end in la[c], lb[c].
// Below 64 lanes per row the slots inside a wave are folded by shuffles.
__device__ __forceinline__ void cp_sum2(double2 a, double2 b, int CP, double2* la, double2* lb) {
    const int RPB = 256 / CP;
    if (CP < 64) {
        for (int off = 32; off >= CP; off >>= 1) {
            a.x += __shfl_xor(a.x, off, kWave); a.y += __shfl_xor(a.y, off, kWave);
            b.x += __shfl_xor(b.x, off, kWave); b.y += __shfl_xor(b.y, off, kWave);
        }
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        if (lane < CP) { la[wave * CP + lane] = a; lb[wave * CP + lane] = b; }
        __syncthreads();
        if ((int)threadIdx.x < CP) {
            const int c = threadIdx.x;
            a = cadd(cadd(la[c], la[CP + c]), cadd(la[2 * CP + c], la[3 * CP + c]));
            b = cadd(cadd(lb[c], lb[CP + c]), cadd(lb[2 * CP + c], lb[3 * CP + c]));
        }
        __syncthreads();
        if ((int)threadIdx.x < CP) { la[threadIdx.x] = a; lb[threadIdx.x] = b; }
        __syncthreads();
        return;
    }
    la[threadIdx.x] = a;
    lb[threadIdx.x] = b;
    for (int w = RPB >> 1; w > 0; w >>= 1) {
        __syncthreads();
        const int slot = threadIdx.x / CP, c = threadIdx.x % CP;
        if (slot < w) {
            la[slot * CP + c] = cadd(la[slot * CP + c], la[(slot + w) * CP + c]);
            lb[slot * CP + c] = cadd(lb[slot * CP + c], lb[(slot + w) * CP + c]);
        }
    }
    __syncthreads();
}

// Fixed-shape tree sum over the nslot row slots of a CP-lane row layout in
// LDS (a[slot * CP + c]); the result for column c ends in a[c].
__device__ __forceinline__ void slot_tree(double2* a, int CP, int nslot) {
    for (int w = nslot >> 1; w > 0; w >>= 1) {
        __syncthreads();
        const int slot = threadIdx.x / CP, c = threadIdx.x % CP;
        if (slot < w) a[slot * CP + c] = cadd(a[slot * CP + c], a[(slot + w) * CP + c]);
    }
    __syncthreads();
}

// --------------------------------------------------------- vector updates
// Thread mapping of the elementwise kernels: CP lanes (power of two >= C)
// per row, 256 / CP rows per pass over a tile.

__device__ __forceinline__ float2 jacobi_z(float2 r, double kd, double md, double wmu) {
    // z = r / (Kd - i wmu Md)
    const double dr = kd, di = -wmu * md;
    const double inv = 1.0 / (dr * dr + di * di);
    return f2((float)(((double)r.x * dr + (double)r.y * di) * inv),
              (float)(((double)r.y * dr - (double)r.x * di) * inv));
}

// D^-1 = 1 / (Kd - i wmu Md) in complex64 for single-column solves (one
// frequency per mesh; a row takes its segment's): the vector kernels then read
// 8 bytes per row instead of Kd, Md.
__global__ void k_dinv(Op op, float2* __restrict__ dinv) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= op.ntiles * kTR) return;
    float2 v = f2(0.f, 0.f);
    if (i < op.nrow_valid) {
        const int seg = op.tile_seg ? op.tile_seg[i / kTR] : 0;
        const double dr = op.Kd[i], di = -op.wmu[seg] * op.Md[i];
        const double inv = 1.0 / (dr * dr + di * di);
        v = f2((float)(dr * inv), (float)(-di * inv));
    }
    dinv[i] = v;
}

// r = (r64 / |r64|) in complex64, x = 0, z = D^-1 r, p = z; partials r^T z,
// |r|^2. dinv (or NULL): the precomputed D^-1 of single-column solves.
__global__ void __launch_bounds__(256)
k_inner_init(Op op, int CP, const double2* __restrict__ R64, const ColState* __restrict__ st,
             const float2* __restrict__ dinv, float2* __restrict__ Xi, float2* __restrict__ R,
             float2* __restrict__ Z, float2* __restrict__ P, double2* __restrict__ p0, double2* __restrict__ p1) {
    __shared__ double2 ra[256], rb[256];
    const int tile = blockIdx.x, C = op.C;
    const int c = threadIdx.x % CP, slot = threadIdx.x / CP, RPB = 256 / CP;
    const int seg = op.tile_seg ? op.tile_seg[tile] : 0;
    double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
    if (c < C) {
        const ColState& S = st[seg * C + c];
        const double inv = S.scale > 0.0 ? 1.0 / S.scale : 0.0;
        const double wmu = op.wmu[seg * C + c];
        for (int r0 = 0; r0 < kTR; r0 += RPB) {
            const int i = tile * kTR + r0 + slot;
            const size_t o = (size_t)i * C + c;
            float2 r = f2(0.f, 0.f), z = f2(0.f, 0.f);
            if (S.outer && i < op.nrow_valid) {
                const double2 rr = R64[o];
                r = f2((float)(rr.x * inv), (float)(rr.y * inv));
                z = dinv ? cmulf(r, dinv[i]) : jacobi_z(r, op.Kd[i], op.Md[i], wmu);
            }
            Xi[o] = f2(0.f, 0.f);
            R[o] = r;
            Z[o] = z;
            P[o] = z;
            a.x += (double)r.x * z.x - (double)r.y * z.y;
            a.y += (double)r.x * z.y + (double)r.y * z.x;
            b.x += (double)r.x * r.x + (double)r.y * r.y;
        }
    }
    cp_sum2(a, b, CP, ra, rb);
    if ((int)threadIdx.x < C && (int)threadIdx.x < CP) {
        p0[(size_t)tile * C + threadIdx.x] = ra[threadIdx.x];
        p1[(size_t)tile * C + threadIdx.x] = rb[threadIdx.x];
    }
}

// r -= alpha q; z = D^-1 r for the active columns; partials of r^T z and
// |r|^2. x += alpha p waits for k_pupdate, which reads p anyway. dinv (or
// NULL): the precomputed D^-1 of single-column solves.
// jac = 0 (SSOR): only r and its |r|^2 partials; z and r^T z follow the sweeps.
__global__ void __launch_bounds__(256)
k_update(Op op, int CP, const ColState* __restrict__ st, float2* __restrict__ R, float2* __restrict__ Z,
         const float2* __restrict__ Q, const float2* __restrict__ dinv, double2* __restrict__ p0,
         double2* __restrict__ p1, int jac) {
    __shared__ double2 ra[256], rb[256];
    const int tile = tile_of(op, blockIdx.x), C = op.C;
    const int c = threadIdx.x % CP, slot = threadIdx.x / CP, RPB = 256 / CP;
    const int seg = op.tile_seg ? op.tile_seg[tile] : 0;
    double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
    if (c < C) {
        const ColState& S = st[seg * C + c];
        if (S.active) {
            const float ax = (float)S.alpha.x, ay = (float)S.alpha.y;
            const double wmu = op.wmu[seg * C + c];
            for (int r0 = 0; r0 < kTR; r0 += RPB) {
                const int i = tile * kTR + r0 + slot;
                if (i >= op.nrow_valid) break;
                const size_t o = (size_t)i * C + c;
                const float2 q = Q[o];
                float2 r = R[o];
                r.x -= ax * q.x - ay * q.y;
                r.y -= ax * q.y + ay * q.x;
                R[o] = r;
                if (jac) {
                    const float2 z = dinv ? cmulf(r, dinv[i]) : jacobi_z(r, op.Kd[i], op.Md[i], wmu);
                    Z[o] = z;
                    a.x += (double)r.x * z.x - (double)r.y * z.y;
                    a.y += (double)r.x * z.y + (double)r.y * z.x;
                }
                b.x += (double)r.x * r.x + (double)r.y * r.y;
            }
        }
    }
    cp_sum2(a, b, CP, ra, rb);
    if ((int)threadIdx.x < C && (int)threadIdx.x < CP) {
        p0[(size_t)tile * C + threadIdx.x] = ra[threadIdx.x];
        p1[(size_t)tile * C + threadIdx.x] = rb[threadIdx.x];
    }
}

// x += alpha p for the columns whose alpha was applied to r this iteration,
// then p = z + beta p for those still active. SQMR (XQ not null): the
// smoothed iterate x_Q = (1 - c^2) x_Q + c^2 x with this step's c^2 (x_Q = 0
// before the first step).
__global__ void __launch_bounds__(256)
k_pupdate(Op op, int CP, const ColState* __restrict__ st, const float2* __restrict__ Z, float2* __restrict__ P,
          float2* __restrict__ Xi, float2* __restrict__ XQ) {
    const int tile = tile_of(op, blockIdx.x), C = op.C;
    const int c = threadIdx.x % CP, slot = threadIdx.x / CP, RPB = 256 / CP;
    if (c >= C) return;
    const int seg = op.tile_seg ? op.tile_seg[tile] : 0;
    const ColState& S = st[seg * C + c];
    if (!S.stepped) return;
    const bool more = S.active;
    const float ax = (float)S.alpha.x, ay = (float)S.alpha.y;
    const float bx = (float)S.beta.x, by = (float)S.beta.y;
    for (int r0 = 0; r0 < kTR; r0 += RPB) {
        const int i = tile * kTR + r0 + slot;
        if (i >= op.nrow_valid) break;
        const size_t o = (size_t)i * C + c;
        const float2 z = Z[o], p = P[o], x = Xi[o];
        const float2 xn = f2(x.x + ax * p.x - ay * p.y, x.y + ax * p.y + ay * p.x);
        Xi[o] = xn;
        if (XQ && S.sqmr) {
            const float cq = (float)S.cq, cp = (float)(1.0 - S.cq);
            const float2 xq = S.kin > 1 ? XQ[o] : f2(0.f, 0.f);
            XQ[o] = f2(cp * xq.x + cq * xn.x, cp * xq.y + cq * xn.y);
        }
        if (more) P[o] = f2(z.x + bx * p.x - by * p.y, z.y + bx * p.y + by * p.x);
    }
}

// ------------------------------------------- multicolour SSOR
// Symmetric successive over-relaxation, the SOR family of the paper's
// single-process runs (Section 5.3, Table 2), made parallel by a multicolour
// ordering: no two DOFs of one colour share a matrix entry, and the sweeps
// take the colours in order, all rows of a colour at once. With D = diag A(w)
// and L, U the entries coupling a row to earlier and to later colours
// (U = L^T: A is complex symmetric), the preconditioner is
//   M = (D / omega + L) (D / omega)^-1 (D / omega + U)
// (the factor (2 - omega) / omega left out: COCG's iterates do not depend on
// a constant scaling of M). z = M^-1 r is the forward sweep
//   y_i = omega (r_i - sum_{j in L(i)} a_ij y_j) / d_i       colours 0 .. nc-1
// then the backward sweep
//   z_i = y_i - omega (sum_{j in U(i)} a_ij z_j) / d_i        colours nc-1 .. 0
// in place in Z. M is complex symmetric, so COCG's short recurrence holds.
// Per column c: a_ij = K_ij - i w_c mu0 M_ij, d_i = Kd_i - i w_c mu0 Md_i.
struct SsorOp {
    const int32_t* row;
    const int32_t* rp;     // L part (forward) or U part (backward)
    const int32_t* col;
    const float* K;
    const float* M;
    const double2* dg;     // {Kd, Md} of each listed row
};

__device__ __forceinline__ void ssor_row_out(double2 kdmd, int i, int C, int c, float2 ak, float2 am, double wmu,
                                             float omega, bool bwd, const float2* __restrict__ R,
                                             float2* __restrict__ Z) {
    // s = sum a_ij v_j = ak - i wmu am; d = Kd - i wmu Md
    const float2 sv = f2(ak.x + (float)wmu * am.y, ak.y - (float)wmu * am.x);
    const double dr = kdmd.x, di = -wmu * kdmd.y;
    const double inv = 1.0 / (dr * dr + di * di);
    const float2 dinv = f2((float)(dr * inv), (float)(-di * inv));
    const size_t o = (size_t)i * C + c;
    if (!bwd) {
        const float2 r = R[o];
        const float2 t = f2(omega * (r.x - sv.x), omega * (r.y - sv.y));
        Z[o] = cmulf(t, dinv);
    } else {
        const float2 y = Z[o];
        const float2 t = cmulf(f2(omega * sv.x, omega * sv.y), dinv);
        Z[o] = f2(y.x - t.x, y.y - t.y);
    }
}

// C <= 4 columns: G lanes share a row's entries (lane l takes entries l,
// l + G, ...), every lane accumulates all CM columns, then a shuffle
// reduction over the G lanes (fixed order). Rows [p0, p1) of the colour
// order. st (or null): columns whose inner solve stopped are skipped.
template <int G, int CM, bool BWD>
__global__ void __launch_bounds__(256)
k_ssor_n(Op op, SsorOp so, int p0, int p1, const ColState* __restrict__ st, const float2* __restrict__ R,
         float2* __restrict__ Z, float omega) {
    constexpr int RPB = 256 / G;
    const int slot = threadIdx.x / G, l = threadIdx.x % G;
    const int p = p0 + blockIdx.x * RPB + slot;
    if (p >= p1) return;   // the whole lane group of this row
    const int C = op.C;
    const int i = so.row[p];
    bool live[CM];
#pragma unroll
    for (int u = 0; u < CM; ++u) live[u] = u < C && (!st || st[u].active);
    float2 ak[CM], am[CM];
#pragma unroll
    for (int u = 0; u < CM; ++u) { ak[u] = f2(0.f, 0.f); am[u] = f2(0.f, 0.f); }
    const int32_t e = so.rp[p + 1];
    for (int32_t k = so.rp[p] + l; k < e; k += G) {
        const int32_t j = so.col[k];
        const float kv = so.K[k], mv = so.M[k];
        const float2* zr = Z + (size_t)j * C;
#pragma unroll
        for (int u = 0; u < CM; ++u) {
            if (!live[u]) continue;
            const float2 v = zr[u];
            ak[u].x += kv * v.x; ak[u].y += kv * v.y;
            am[u].x += mv * v.x; am[u].y += mv * v.y;
        }
    }
#pragma unroll
    for (int off = G >> 1; off > 0; off >>= 1)
#pragma unroll
        for (int u = 0; u < CM; ++u) {
            ak[u].x += __shfl_xor(ak[u].x, off, G); ak[u].y += __shfl_xor(ak[u].y, off, G);
            am[u].x += __shfl_xor(am[u].x, off, G); am[u].y += __shfl_xor(am[u].y, off, G);
        }
    // lane u writes column u (every lane holds the same sums)
#pragma unroll
    for (int u = 0; u < CM; ++u)
        if (l == u && live[u]) ssor_row_out(so.dg[p], i, C, u, ak[u], am[u], op.wmu[u], omega, BWD, R, Z);
}

// More columns: LPR lanes per row, CPL consecutive columns per lane; the
// row's entries are loaded across the lanes and handed out by shuffles, all
// of a chunk's gathers in flight at once (as k_spmm_g).
template <int LPR, int CPL, bool BWD>
__global__ void __launch_bounds__(256)
k_ssor_c(Op op, SsorOp so, int p0, int p1, const ColState* __restrict__ st, const float2* __restrict__ R,
         float2* __restrict__ Z, float omega) {
    constexpr int RPB = 256 / LPR;
    constexpr int NB = 12;                        // entries per trip (an L or U part has 3..10)
    constexpr int NH = (NB + LPR - 1) / LPR;
    const int slot = threadIdx.x / LPR, l = threadIdx.x % LPR;
    const int p = p0 + blockIdx.x * RPB + slot;
    if (p >= p1) return;   // the whole lane group of this row
    const int C = op.C;
    const int i = so.row[p];
    const double2 dgp = so.dg[p];
    bool live[CPL];
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
        const int c = l * CPL + u;
        live[u] = c < C && (!st || st[c].active);
    }
    float2 ak[CPL], am[CPL];
#pragma unroll
    for (int u = 0; u < CPL; ++u) { ak[u] = f2(0.f, 0.f); am[u] = f2(0.f, 0.f); }
    const int32_t ke = so.rp[p + 1];
    for (int32_t kb = so.rp[p]; kb < ke; kb += NB) {
        int32_t cj[NH];
        float kv[NH], mv[NH];
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            const int32_t k = kb + h * LPR + l;
            const bool ok = h * LPR + l < NB && k < ke;
            cj[h] = ok ? so.col[k] : 0;
            kv[h] = ok ? so.K[k] : 0.f;
            mv[h] = ok ? so.M[k] : 0.f;
        }
        float2 xv[NB][CPL];
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int j = __shfl(cj[q / LPR], q % LPR, LPR);
            const bool ok = kb + q < ke;
            const float2* zr = Z + (size_t)j * C + l * CPL;
#pragma unroll
            for (int u = 0; u < CPL; ++u) xv[q][u] = (ok && live[u]) ? zr[u] : f2(0.f, 0.f);
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const float kq = __shfl(kv[q / LPR], q % LPR, LPR);
            const float mq = __shfl(mv[q / LPR], q % LPR, LPR);
#pragma unroll
            for (int u = 0; u < CPL; ++u) {
                ak[u].x += kq * xv[q][u].x; ak[u].y += kq * xv[q][u].y;
                am[u].x += mq * xv[q][u].x; am[u].y += mq * xv[q][u].y;
            }
        }
    }
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
        const int c = l * CPL + u;
        if (live[u]) ssor_row_out(dgp, i, C, c, ak[u], am[u], op.wmu[c], omega, BWD, R, Z);
    }
}

// Eisenstat's form of the SSOR-preconditioned COCG (many columns). With
// D~ = D / omega, L1 = D~ + L and U1 = D~ + U = L1^T, the iteration runs on
// the split system  L1^-1 A U1^-1 (scaled by D~^1/2 on both sides, which
// keeps it complex symmetric and equal to COCG with M = L1 D~^-1 U1), and
// A = L1 + U1 + (D - 2 D~) turns its product into the two triangular solves:
//   t = U1^-1 p     (the U sweep, colours nc-1 .. 0: the forward formula on
//                    the U entries)
//   y = L1^-1 (p + (D - 2 D~) t)          (this kernel, colours 0 .. nc-1)
//   q = t + y       (the product with the split operator, never formed)
// In the variables used here (p = D~^1/2 p^, r = D~^1/2 r^) the scalars are
//   p^T q, rho = r^T D~^-1 r, r -= alpha D~ q, x += alpha t, p = r + beta p,
// and x is the correction itself (the sum of alpha U1^-1 p). This kernel also
// leaves the block's partial sums of p^T (t + y), column c's at part[c * cs +
// base + block] (rows of a colour: no early exit, every thread reaches the
// barrier).
template <int LPR, int CPL>
__global__ void __launch_bounds__(256)
k_ssor_eis(Op op, SsorOp so, int p0, int p1, const ColState* __restrict__ st, const float2* __restrict__ P,
           const float2* __restrict__ T, float2* __restrict__ Y, float omega, double2* __restrict__ part,
           int base, int64_t cs) {
    constexpr int RPB = 256 / LPR;
    constexpr int NB = 12;
    constexpr int NH = (NB + LPR - 1) / LPR;
    __shared__ double2 red[RPB][LPR * CPL];
    const int slot = threadIdx.x / LPR, l = threadIdx.x % LPR;
    const int C = op.C;
    const float cdt = 1.f - 2.f / omega;   // (D - 2 D~) = (1 - 2 / omega) D
    bool colok[CPL];
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
        const int c = l * CPL + u;
        colok[u] = c < C && (!st || st[c].active);
    }
    double2 pa[CPL];
#pragma unroll
    for (int u = 0; u < CPL; ++u) pa[u] = make_double2(0.0, 0.0);
    // the block strides over the colour's rows (few blocks: few partial slots
    // for the alpha reduction); the loop bound is the same for all its threads
    for (int pb = p0 + blockIdx.x * RPB; pb < p1; pb += gridDim.x * RPB) {
        const int p = pb + slot;
        const bool rowok = p < p1;   // a whole lane group of this row
        const int i = rowok ? so.row[p] : 0;
        bool live[CPL];
#pragma unroll
        for (int u = 0; u < CPL; ++u) live[u] = rowok && colok[u];
        float2 ak[CPL], am[CPL];
#pragma unroll
        for (int u = 0; u < CPL; ++u) { ak[u] = f2(0.f, 0.f); am[u] = f2(0.f, 0.f); }
        const int32_t ke = rowok ? so.rp[p + 1] : 0;
        for (int32_t kb = rowok ? so.rp[p] : 0; kb < ke; kb += NB) {
            int32_t cj[NH];
            float kv[NH], mv[NH];
#pragma unroll
            for (int h = 0; h < NH; ++h) {
                const int32_t k = kb + h * LPR + l;
                const bool ok = h * LPR + l < NB && k < ke;
                cj[h] = ok ? so.col[k] : 0;
                kv[h] = ok ? so.K[k] : 0.f;
                mv[h] = ok ? so.M[k] : 0.f;
            }
            float2 xv[NB][CPL];
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                const int j = __shfl(cj[q / LPR], q % LPR, LPR);
                const bool ok = kb + q < ke;
                const float2* yr = Y + (size_t)j * C + l * CPL;
#pragma unroll
                for (int u = 0; u < CPL; ++u) xv[q][u] = (ok && live[u]) ? yr[u] : f2(0.f, 0.f);
            }
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                const float kq = __shfl(kv[q / LPR], q % LPR, LPR);
                const float mq = __shfl(mv[q / LPR], q % LPR, LPR);
#pragma unroll
                for (int u = 0; u < CPL; ++u) {
                    ak[u].x += kq * xv[q][u].x; ak[u].y += kq * xv[q][u].y;
                    am[u].x += mq * xv[q][u].x; am[u].y += mq * xv[q][u].y;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < CPL; ++u) {
            if (!live[u]) continue;
            const int c = l * CPL + u;
            const double wmu = op.wmu[c];
            // s = sum a_ij y_j = ak - i wmu am; d = Kd - i wmu Md
            const float2 sv = f2(ak[u].x + (float)wmu * am[u].y, ak[u].y - (float)wmu * am[u].x);
            const double2 kdmd = so.dg[p];
            const double dr = kdmd.x, di = -wmu * kdmd.y;
            const double inv = 1.0 / (dr * dr + di * di);
            const float2 dinv = f2((float)(dr * inv), (float)(-di * inv));
            const size_t o = (size_t)i * C + c;
            const float2 pv = P[o], tv = T[o];
            const float2 dt = cmulf(f2((float)dr, (float)di), tv);
            const float2 rhs = f2(pv.x + cdt * dt.x - sv.x, pv.y + cdt * dt.y - sv.y);
            const float2 y = cmulf(f2(omega * rhs.x, omega * rhs.y), dinv);
            Y[o] = y;
            const float2 qv = f2(tv.x + y.x, tv.y + y.y);
            pa[u].x += (double)pv.x * qv.x - (double)pv.y * qv.y;
            pa[u].y += (double)pv.x * qv.y + (double)pv.y * qv.x;
        }
    }
#pragma unroll
    for (int u = 0; u < CPL; ++u) red[slot][l * CPL + u] = pa[u];
    __syncthreads();
    for (int c = threadIdx.x; c < C && c < LPR * CPL; c += 256) {
        double2 a = make_double2(0.0, 0.0);
        for (int r = 0; r < RPB; ++r) a = cadd(a, red[r][c]);
        part[(size_t)c * cs + base + blockIdx.x] = a;
    }
}

// The Eisenstat U pass with the direction update folded in: for a column
// whose beta step ran (stepped) and that is still active, p = r + beta p at
// the row first (written back: the L pass reads it), then t = omega (p - s)/d
// with s over the row's U entries (gathered from T), colours descending.
template <int LPR, int CPL>
__global__ void __launch_bounds__(256)
k_ssor_eis_u(Op op, SsorOp so, int p0, int p1, const ColState* __restrict__ st, const float2* __restrict__ R,
             float2* __restrict__ P, float2* __restrict__ T, float omega) {
    constexpr int RPB = 256 / LPR;
    constexpr int NB = 12;
    constexpr int NH = (NB + LPR - 1) / LPR;
    const int slot = threadIdx.x / LPR, l = threadIdx.x % LPR;
    const int p = p0 + blockIdx.x * RPB + slot;
    if (p >= p1) return;   // the whole lane group of this row
    const int C = op.C;
    const int i = so.row[p];
    const double2 dgp = so.dg[p];
    bool live[CPL];
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
        const int c = l * CPL + u;
        live[u] = c < C && st[c].active;
    }
    float2 ak[CPL], am[CPL];
#pragma unroll
    for (int u = 0; u < CPL; ++u) { ak[u] = f2(0.f, 0.f); am[u] = f2(0.f, 0.f); }
    const int32_t ke = so.rp[p + 1];
    for (int32_t kb = so.rp[p]; kb < ke; kb += NB) {
        int32_t cj[NH];
        float kv[NH], mv[NH];
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            const int32_t k = kb + h * LPR + l;
            const bool ok = h * LPR + l < NB && k < ke;
            cj[h] = ok ? so.col[k] : 0;
            kv[h] = ok ? so.K[k] : 0.f;
            mv[h] = ok ? so.M[k] : 0.f;
        }
        float2 xv[NB][CPL];
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int j = __shfl(cj[q / LPR], q % LPR, LPR);
            const bool ok = kb + q < ke;
            const float2* tr = T + (size_t)j * C + l * CPL;
#pragma unroll
            for (int u = 0; u < CPL; ++u) xv[q][u] = (ok && live[u]) ? tr[u] : f2(0.f, 0.f);
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const float kq = __shfl(kv[q / LPR], q % LPR, LPR);
            const float mq = __shfl(mv[q / LPR], q % LPR, LPR);
#pragma unroll
            for (int u = 0; u < CPL; ++u) {
                ak[u].x += kq * xv[q][u].x; ak[u].y += kq * xv[q][u].y;
                am[u].x += mq * xv[q][u].x; am[u].y += mq * xv[q][u].y;
            }
        }
    }
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
        const int c = l * CPL + u;
        if (!live[u]) continue;
        const ColState& S = st[c];
        const size_t o = (size_t)i * C + c;
        float2 pv = P[o];
        if (S.stepped) {
            const float bx = (float)S.beta.x, by = (float)S.beta.y;
            const float2 rv = R[o];
            pv = f2(rv.x + bx * pv.x - by * pv.y, rv.y + bx * pv.y + by * pv.x);
            P[o] = pv;
        }
        const double wmu = op.wmu[c];
        const float2 sv = f2(ak[u].x + (float)wmu * am[u].y, ak[u].y - (float)wmu * am[u].x);
        const double dr = dgp.x, di = -wmu * dgp.y;
        const double inv = 1.0 / (dr * dr + di * di);
        const float2 dinv = f2((float)(dr * inv), (float)(-di * inv));
        const float2 t = cmulf(f2(omega * (pv.x - sv.x), omega * (pv.y - sv.y)), dinv);
        T[o] = t;
    }
}

// Start of an Eisenstat inner solve, after y = L1^-1 r0 (the forward sweep
// into Y): r = D~ y, p = r; partials r^T y (= r^T D~^-1 r, rho) and
// sum |r_i|^2 / |D~_i| (the squared norm of the split residual).
__global__ void __launch_bounds__(256)
k_eis_init(Op op, int CP, const ColState* __restrict__ st, const float2* __restrict__ Y, float2* __restrict__ R,
           float2* __restrict__ P, float omega, double2* __restrict__ p0, double2* __restrict__ p1) {
    __shared__ double2 ra[256], rb[256];
    const int tile = blockIdx.x, C = op.C;
    const int c = threadIdx.x % CP, slot = threadIdx.x / CP, RPB = 256 / CP;
    double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
    if (c < C && st[c].outer) {
        const double wmu = op.wmu[c];
        for (int r0 = 0; r0 < kTR; r0 += RPB) {
            const int i = tile * kTR + r0 + slot;
            if (i >= op.nrow_valid) break;
            const size_t o = (size_t)i * C + c;
            const double dr = op.Kd[i] / omega, di = -wmu * op.Md[i] / omega;   // D~
            const float2 y = Y[o];
            const float2 r = cmulf(f2((float)dr, (float)di), y);
            R[o] = r;
            P[o] = r;
            a.x += (double)r.x * y.x - (double)r.y * y.y;
            a.y += (double)r.x * y.y + (double)r.y * y.x;
            b.x += ((double)r.x * r.x + (double)r.y * r.y) / sqrt(dr * dr + di * di);
        }
    }
    cp_sum2(a, b, CP, ra, rb);
    if ((int)threadIdx.x < C && (int)threadIdx.x < CP) {
        p0[(size_t)tile * C + threadIdx.x] = ra[threadIdx.x];
        p1[(size_t)tile * C + threadIdx.x] = rb[threadIdx.x];
    }
}

// The Eisenstat step after alpha: x += alpha t, r -= alpha D~ (t + y);
// partials rho' = r^T D~^-1 r and sum |r_i|^2 / |D~_i|, column by column
// (column c's of tile t at c * ntiles + t). SQMR (XQ not null): first the
// smoothing step of the previous beta step, x_Q = (1 - c^2) x_Q + c^2 x.
__global__ void __launch_bounds__(256)
k_eis_update(Op op, int CP, const ColState* __restrict__ st, const float2* __restrict__ T,
             const float2* __restrict__ Y, float2* __restrict__ R, float2* __restrict__ Xi,
             float2* __restrict__ XQ, float omega, double2* __restrict__ p0, double2* __restrict__ p1) {
    const int64_t cs = op.ntiles;   // the partials column by column
    __shared__ double2 ra[256], rb[256];
    const int tile = tile_of(op, blockIdx.x), C = op.C;
    const int c = threadIdx.x % CP, slot = threadIdx.x / CP, RPB = 256 / CP;
    double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
    if (c < C && st[c].active) {
        const ColState& S = st[c];
        const float ax = (float)S.alpha.x, ay = (float)S.alpha.y;
        const double wmu = op.wmu[c];
        // SQMR: x is the iterate of the latest beta step, whose c^2 the state
        // holds; x_Q takes that step here, before x moves on (the last step
        // of an inner solve is taken by k_ir_update)
        const bool smooth = XQ && S.sqmr && S.kin > 0;
        const float cq = (float)S.cq, cp = (float)(1.0 - S.cq);
        for (int r0 = 0; r0 < kTR; r0 += RPB) {
            const int i = tile * kTR + r0 + slot;
            if (i >= op.nrow_valid) break;
            const size_t o = (size_t)i * C + c;
            const double dr = op.Kd[i] / omega, di = -wmu * op.Md[i] / omega;   // D~
            const double inv = 1.0 / (dr * dr + di * di);
            const float2 t = T[o], y = Y[o];
            float2 x = Xi[o];
            if (smooth) {
                const float2 xq = S.kin > 1 ? XQ[o] : f2(0.f, 0.f);
                XQ[o] = f2(cp * xq.x + cq * x.x, cp * xq.y + cq * x.y);
            }
            x.x += ax * t.x - ay * t.y;
            x.y += ax * t.y + ay * t.x;
            Xi[o] = x;
            const float2 q = cmulf(f2((float)dr, (float)di), f2(t.x + y.x, t.y + y.y));   // D~ (t + y)
            float2 r = R[o];
            r.x -= ax * q.x - ay * q.y;
            r.y -= ax * q.y + ay * q.x;
            R[o] = r;
            const float2 z = cmulf(r, f2((float)(dr * inv), (float)(-di * inv)));   // D~^-1 r
            a.x += (double)r.x * z.x - (double)r.y * z.y;
            a.y += (double)r.x * z.y + (double)r.y * z.x;
            b.x += ((double)r.x * r.x + (double)r.y * r.y) * sqrt(inv);
        }
    }
    cp_sum2(a, b, CP, ra, rb);
    if ((int)threadIdx.x < C && (int)threadIdx.x < CP) {
        p0[(size_t)threadIdx.x * cs + tile] = ra[threadIdx.x];
        p1[(size_t)threadIdx.x * cs + tile] = rb[threadIdx.x];
    }
}


// {Kd, Md} of each listed row of the multicolour order
__global__ void k_ssor_dg(int n, const int32_t* __restrict__ row, const double* __restrict__ Kd,
                          const double* __restrict__ Md, double2* __restrict__ dg) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    dg[p] = make_double2(Kd[row[p]], Md[row[p]]);
}

// Partials of r^T z per tile and column (the sweeps wrote z); with P not
// null also p = z (the start of an inner solve). st (or null) as above; with
// P, columns still in the refinement (outer) take part.
__global__ void __launch_bounds__(256)
k_rz(Op op, int CP, const ColState* __restrict__ st, const float2* __restrict__ R, const float2* __restrict__ Z,
     float2* __restrict__ P, double2* __restrict__ part) {
    __shared__ double2 ra[256], rb[256];
    const int tile = tile_of(op, blockIdx.x), C = op.C;
    const int c = threadIdx.x % CP, slot = threadIdx.x / CP, RPB = 256 / CP;
    double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
    if (c < C && (!st || (P ? st[c].outer : st[c].active))) {
        for (int r0 = 0; r0 < kTR; r0 += RPB) {
            const int i = tile * kTR + r0 + slot;
            if (i >= op.nrow_valid) break;
            const size_t o = (size_t)i * C + c;
            const float2 r = R[o], z = Z[o];
            if (P) P[o] = z;
            a.x += (double)r.x * z.x - (double)r.y * z.y;
            a.y += (double)r.x * z.y + (double)r.y * z.x;
        }
    }
    cp_sum2(a, b, CP, ra, rb);
    if ((int)threadIdx.x < C && (int)threadIdx.x < CP) part[(size_t)tile * C + threadIdx.x] = ra[threadIdx.x];
}

__global__ void k_ssor_vals(int64_t n, const int32_t* __restrict__ pos, const float* __restrict__ K,
                            const float* __restrict__ M, float* __restrict__ oK, float* __restrict__ oM) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    const int32_t k = pos[e];
    oK[e] = K[k];
    oM[e] = M[k];
}

// ------------------------------------------- reductions in the consumers
// For one mesh whose partials are few, every block of the next vector kernel
// sums them itself (the same fixed order in every block, so all blocks agree
// bitwise) instead of a reduction kernel running in between: the iteration is
// the SpMM, the update (which forms alpha first) and the direction update
// (which tests convergence and forms beta first). Each kernel reads the
// column state from one slot and its first block writes the advanced state to
// the other slot, so no block reads a value another block of the same launch
// may be writing. The two vector kernels take tpb tiles per block (fewer
// blocks, fewer partials for the next consumer) and one partial slot per
// block. (Folding the direction update into the SpMM, gathering an
// interleaved {z, p}, measured slower than this arrangement.)

// Sums over the partial slots [0, nslot) of every column, by all 256 threads
// (thread t takes column t % CP); column c's sums end in la[c], lb[c].
__device__ __forceinline__ void cols_sum2(const double2* __restrict__ p0, const double2* __restrict__ p1, int nslot,
                                          int C, int CP, double2* la, double2* lb) {
    const int c = threadIdx.x % CP, slot = threadIdx.x / CP, RPB = 256 / CP;
    double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
    if (c < C) {
        // eight loads in flight, then the additions in the same order
        for (int e0 = slot; e0 < nslot; e0 += 8 * RPB) {
            double2 va[8], vb[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = e0 + u * RPB;
                va[u] = e < nslot ? p0[(size_t)e * C + c] : make_double2(0.0, 0.0);
                vb[u] = (p1 && e < nslot) ? p1[(size_t)e * C + c] : make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                a = cadd(a, va[u]);
                b = cadd(b, vb[u]);
            }
        }
    }
    cp_sum2(a, b, CP, la, lb);
}

// alpha from the nps SpMM partials of p^T q (state slot s1 -> s0), then over
// tpb tiles: r -= alpha q; z = D^-1 r; partials r^T z, |r|^2 (one slot per
// block). x += alpha p waits for k_pupdate_p, which reads p anyway. dinv (or
// NULL): the precomputed D^-1 of a single-column solve.
__global__ void __launch_bounds__(256)
k_update_p(Op op, int CP, int tpb, const ColState* __restrict__ s1, ColState* __restrict__ s0,
           const double2* __restrict__ ps, int nps, float2* __restrict__ R, float2* __restrict__ Z,
           const float2* __restrict__ Q, const float2* __restrict__ dinv, double2* __restrict__ p0,
           double2* __restrict__ p1) {
    __shared__ double2 ra[256], rb[256];
    const int C = op.C;
    const int c = threadIdx.x % CP, slot = threadIdx.x / CP, RPB = 256 / CP;
    const int i0 = blockIdx.x * tpb * kTR, i1 = min(i0 + tpb * kTR, op.nrow_valid);
    const int cc = min(c, C - 1);   // lanes past the last column load column C-1 and store nothing
    // The first four rows' vectors and the two scalars the update needs are
    // loaded ahead of the partial sums (none of them depends on alpha).
    float2 q[4], r[4], dv[4];
    double kd[4], md[4];
    auto load4 = [&](int ib) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = max(min(ib + u * RPB, i1 - 1), 0);   // in range; the duplicates are not stored
            const size_t o = (size_t)i * C + cc;
            q[u] = Q[o]; r[u] = R[o];
            if (dinv) dv[u] = dinv[i];
            else { kd[u] = op.Kd[i]; md[u] = op.Md[i]; }
        }
    };
    load4(i0 + slot);
    const int act0 = s1[cc].active;
    const double2 rho = s1[cc].rho;
    cols_sum2(ps, nullptr, nps, C, CP, ra, rb);
    bool act = false;
    double2 alpha = make_double2(0.0, 0.0);
    if (c < C) {
        const double2 pq = ra[c];
        act = act0 && cfinite(pq) && !czero(pq);
        if (act) alpha = cdiv(rho, pq);
        if (blockIdx.x == 0 && slot == 0) {
            ColState S = s1[c];
            if (S.active) step_alpha(S, pq);
            s0[c] = S;
        }
    }
    __syncthreads();   // ra is reused below
    double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
    if (act) {
        const float ax = (float)alpha.x, ay = (float)alpha.y;
        const double wmu = op.wmu[c];
        for (int ib = i0 + slot; ib < i1; ib += 4 * RPB) {
            if (ib != i0 + slot) load4(ib);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = ib + u * RPB;
                if (i >= i1) break;
                const size_t o = (size_t)i * C + c;
                r[u].x -= ax * q[u].x - ay * q[u].y;
                r[u].y -= ax * q[u].y + ay * q[u].x;
                const float2 z = dinv ? cmulf(r[u], dv[u]) : jacobi_z(r[u], kd[u], md[u], wmu);
                R[o] = r[u];
                Z[o] = z;
                a.x += (double)r[u].x * z.x - (double)r[u].y * z.y;
                a.y += (double)r[u].x * z.y + (double)r[u].y * z.x;
                b.x += (double)r[u].x * r[u].x + (double)r[u].y * r[u].y;
            }
        }
    }
    cp_sum2(a, b, CP, ra, rb);
    if ((int)threadIdx.x < C && (int)threadIdx.x < CP) {
        p0[(size_t)blockIdx.x * C + threadIdx.x] = ra[threadIdx.x];
        p1[(size_t)blockIdx.x * C + threadIdx.x] = rb[threadIdx.x];
    }
}

// convergence test and beta from the npu partials of r^T z and |r|^2 (state
// slot s0 -> s1); then, over tpb tiles, for the columns whose alpha was
// applied to r: x += alpha p, and for those still active: p = z + beta p.
__global__ void __launch_bounds__(256)
k_pupdate_p(Op op, int CP, int tpb, const ColState* __restrict__ s0, ColState* __restrict__ s1,
            const double2* __restrict__ pg, const double2* __restrict__ pr, int npu, const float2* __restrict__ Z,
            float2* __restrict__ P, float2* __restrict__ Xi) {
    __shared__ double2 ra[256], rb[256];
    const int C = op.C;
    const int c = threadIdx.x % CP, slot = threadIdx.x / CP, RPB = 256 / CP;
    const int i0 = blockIdx.x * tpb * kTR, i1 = min(i0 + tpb * kTR, op.nrow_valid);
    const int cc = min(c, C - 1);   // lanes past the last column load column C-1 and store nothing
    // the first four rows of z, p and x are loaded ahead of the partial sums
    float2 z[4], p[4], x[4];
    auto load4 = [&](int ib) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const size_t o = (size_t)max(min(ib + u * RPB, i1 - 1), 0) * C + cc;   // duplicates are not stored
            z[u] = Z[o];
            p[u] = P[o];
            x[u] = Xi[o];
        }
    };
    load4(i0 + slot);
    cols_sum2(pg, pr, npu, C, CP, ra, rb);
    // one thread per column takes the beta step and hands the scalars to the
    // block through LDS
    __shared__ double2 sab[256][2];
    __shared__ int sflag[256];
    if (slot == 0 && c < C) {
        ColState S = s0[c];
        const bool stepped = S.active;   // this iteration's alpha was applied to r
        if (S.active) step_beta(S, ra[c], rb[c].x);
        if (blockIdx.x == 0) s1[c] = S;
        sab[c][0] = S.alpha;
        sab[c][1] = S.beta;
        sflag[c] = (stepped ? 1 : 0) | (S.active ? 2 : 0);
    }
    __syncthreads();
    if (c >= C) return;
    const int flag = sflag[c];
    if (!(flag & 1)) return;
    const bool more = (flag & 2) != 0;
    const double2 al = sab[c][0], be = sab[c][1];
    const float ax = (float)al.x, ay = (float)al.y;
    const float bx = (float)be.x, by = (float)be.y;
    for (int ib = i0 + slot; ib < i1; ib += 4 * RPB) {
        if (ib != i0 + slot) load4(ib);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = ib + u * RPB;
            if (i >= i1) break;
            const size_t o = (size_t)i * C + c;
            Xi[o] = f2(x[u].x + ax * p[u].x - ay * p[u].y, x[u].y + ax * p[u].y + ay * p[u].x);
            if (more) P[o] = f2(z[u].x + bx * p[u].x - by * p[u].y, z[u].y + bx * p[u].y + by * p[u].x);
        }
    }
}

// The scalar step of the fused step for one column, from the five sums t:
// the product's p^T q, q^T D^-1 r, q^T D^-1 q and the previous step's r^T z,
// |r|^2. kin == 0 (just started): rho and |r|^2 are the state's own;
// otherwise the convergence test (with the stagnation guard) runs first.
__device__ __forceinline__ void fused_scalars(ColState& S, const double2* t) {
    if (S.active && S.kin > 0) {   // the r left by the previous step
        const double2 rz = t[3];
        const double r2 = t[4].x;
        S.rn2 = r2;
        if (!isfinite(r2) || !cfinite(rz)) {
            S.active = 0;
            S.breakdown = 1;
        } else if (r2 <= S.inner_tol2) {
            S.active = 0;
        } else if (stalled_now(S, r2)) {
            S.active = 0;
            S.stalled += 1;
        } else if (relaxed_now(S, r2)) {
            S.active = 0;
        } else if (plateau_now(S, r2)) {
            S.active = 0;
            S.stalled += 1;
        } else if (czero(rz)) {
            S.active = 0;
            S.breakdown = 1;
        } else {
            S.rho = rz;
        }
    }
    if (S.active) {
        const double2 pq = t[0];
        if (!cfinite(pq) || czero(pq)) {
            S.active = 0;
            S.breakdown = 1;
        } else {
            const double2 al = cdiv(S.rho, pq);
            // rho - 2 alpha q^T D^-1 r + alpha^2 q^T D^-1 q
            const double2 next =
                cadd(cadd(S.rho, cscale(cmul(al, t[1]), -2.0)), cmul(cmul(al, al), t[2]));
            const double2 be = cdiv(next, S.rho);
            if (!cfinite(be)) {
                S.active = 0;
                S.breakdown = 1;
            } else {
                S.alpha = al;
                S.beta = be;
                S.iters += 1;
                S.kin += 1;
            }
        }
    }
}

// ------------------------------------------- fused single-column step
// One mesh, one column, D^-1 precomputed: after the product q = A p a single
// vector kernel takes the whole COCG step. The next rho is known before r is
// updated, by expanding
//   (r - alpha q)^T D^-1 (r - alpha q) = rho - 2 alpha q^T D^-1 r + alpha^2 q^T D^-1 q
// with the product's partials, so beta is known too: r -= alpha q,
// z = D^-1 r, x += alpha p and p = z + beta p go in one pass over the rows
// (64 B per row instead of 80 B in two kernels). The exact r^T z and |r|^2
// of the new r are summed at the next step, which tests convergence on them
// and takes that r^T z for its alpha, so the expansion only ever sets beta.
// The iteration is two kernels: the product and this step.
//
// The step (state slot sin -> sout): every block sums the product's nps
// partial triples (three planes of nps) and the previous step's npg partial
// pairs in a fixed order, with all of a thread's loads in flight at once;
// one thread then takes the scalar step (block 0 stores the state) and
// hands alpha and beta to the block; then, over NR tiles, the row updates,
// with the partials of the new r^T z and |r|^2 (one slot per block) into go,
// ro, which must not be pg, pr: other blocks may still be reading those.
// kin == 0 (just started): rho and |r|^2 are the state's own; otherwise the
// convergence test runs first on the previous step's sums. (With the scalar
// step taken by every thread on its own copy of the state, the kernel took
// 19 us instead of 11.)
// snap (or null): a ring of kSnapRing host-memory slots; block 0 also copies
// the new state into slot *gcount and advances the count (the last step of
// every iteration group does, so the host reads the state of a group without
// a copy of its own on the stream).
template <int NR>
__global__ void __launch_bounds__(256)
k_step1(Op op, const ColState* __restrict__ sin, ColState* __restrict__ sout,
        const double2* __restrict__ ps, int nps, const double2* __restrict__ pg, const double2* __restrict__ pr,
        int npg, float2* __restrict__ R, const float2* __restrict__ Q,
        const float2* __restrict__ dinv, float2* __restrict__ P, float2* __restrict__ Xi, double2* __restrict__ go,
        double2* __restrict__ ro, ColState* __restrict__ snap, int* __restrict__ gcount) {
    __shared__ double2 ra[256], rb[256];
    __shared__ double2 scal[3];
    __shared__ double2 tot[5];
    __shared__ ColState s_in;
    static_assert(sizeof(ColState) % 8 == 0 && sizeof(ColState) / 8 <= 256, "state copied as doubles");
    // the state (written by the previous step's block 0) is copied to LDS
    // first, so its load overlaps the partial sums instead of following them
    if (threadIdx.x < sizeof(ColState) / 8)
        reinterpret_cast<double*>(&s_in)[threadIdx.x] = reinterpret_cast<const double*>(sin)[threadIdx.x];
    // NR tiles per block, one row of each per thread: all NR rows of every
    // vector are loaded ahead of the sums
    const int i0 = blockIdx.x * NR * kTR + (int)threadIdx.x, i1 = op.nrow_valid;
    float2 q[NR], r[NR], dv[NR], x[NR], p[NR];
#pragma unroll
    for (int u = 0; u < NR; ++u) {
        const int i = max(min(i0 + u * 256, i1 - 1), 0);   // in range; the duplicates are not stored
        q[u] = Q[i]; r[u] = R[i]; dv[u] = dinv[i]; x[u] = Xi[i]; p[u] = P[i];
    }
    // fixed-order sums of the product's partials (three per tile) and of the
    // previous step's (two per block): strided per thread, then the waves
    {
        double2 v[5];
#pragma unroll
        for (int j = 0; j < 5; ++j) v[j] = make_double2(0.0, 0.0);
        // eight slots of each source per thread in flight (one round up to
        // 2,048 product tiles), then the additions in slot order
        for (int e0 = threadIdx.x; e0 < nps; e0 += 8 * 256) {
            double2 a[8][3];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = e0 + u * 256;
#pragma unroll
                for (int j = 0; j < 3; ++j) a[u][j] = e < nps ? ps[(size_t)j * nps + e] : make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
#pragma unroll
                for (int j = 0; j < 3; ++j) v[j] = cadd(v[j], a[u][j]);
        }
        for (int e0 = threadIdx.x; e0 < npg; e0 += 4 * 256) {
            double2 a[4][2];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = e0 + u * 256;
                a[u][0] = e < npg ? pg[e] : make_double2(0.0, 0.0);
                a[u][1] = e < npg ? pr[e] : make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                v[3] = cadd(v[3], a[u][0]);
                v[4] = cadd(v[4], a[u][1]);
            }
        }
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            const double sx = wave_sum(v[j].x), sy = wave_sum(v[j].y);
            if (lane == 0) ra[wave * 5 + j] = make_double2(sx, sy);
        }
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        const int j = threadIdx.x;
        tot[j] = cadd(cadd(ra[j], ra[5 + j]), cadd(ra[10 + j], ra[15 + j]));
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        ColState S = s_in;
        fused_scalars(S, tot);
        if (blockIdx.x == 0) {
            sout[0] = S;
            if (snap) {
                const int g = *gcount;
                snap[g & (kSnapRing - 1)] = S;
                *gcount = g + 1;
            }
        }
        scal[0] = S.alpha;
        scal[1] = S.beta;
        scal[2] = make_double2(S.active ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    if (scal[2].x == 0.0) return;   // the same in every thread
    const double2 alpha = scal[0], beta = scal[1];
    const float ax = (float)alpha.x, ay = (float)alpha.y, bx = (float)beta.x, by = (float)beta.y;
    double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
    {
#pragma unroll
        for (int u = 0; u < NR; ++u) {
            const int i = i0 + u * 256;
            if (i >= i1) break;
            float2 rr = r[u];
            rr.x -= ax * q[u].x - ay * q[u].y;
            rr.y -= ax * q[u].y + ay * q[u].x;
            const float2 z = cmulf(rr, dv[u]);
            R[i] = rr;
            Xi[i] = f2(x[u].x + ax * p[u].x - ay * p[u].y, x[u].y + ax * p[u].y + ay * p[u].x);
            P[i] = f2(z.x + bx * p[u].x - by * p[u].y, z.y + bx * p[u].y + by * p[u].x);
            a.x += (double)rr.x * z.x - (double)rr.y * z.y;
            a.y += (double)rr.x * z.y + (double)rr.y * z.x;
            b.x += (double)rr.x * rr.x + (double)rr.y * rr.y;
        }
    }
    cp_sum2(a, b, 1, ra, rb);
    if (threadIdx.x == 0) {
        go[blockIdx.x] = ra[0];
        ro[blockIdx.x] = rb[0];
    }
}

// ------------------------------------------- fused step, several meshes
// The fused step for one column per mesh when the meshes' partials are too
// many for every block to sum (an uneven batch, or one large mesh): the
// product (one 256-row tile per block, D^-1 from the double-precision
// diagonal), one block per mesh forming its scalars, then the row update.
// Three kernels per iteration instead of five. Partials are per tile: the
// product's three in planes of ntiles, the step's two in p1, p2.
template <int U>
__global__ void __launch_bounds__(256)
k_spmm_spbs(Op op, const ColState* __restrict__ st, const float2* __restrict__ X, float2* __restrict__ Y,
            const float2* __restrict__ R, double2* __restrict__ partial) {
    __shared__ double2 red[4][3];
    const int tile = tile_of(op, xcd_block(blockIdx.x, gridDim.x));
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int sl = tile * 4 + wave;
    const int seg = op.tile_seg ? op.tile_seg[tile] : 0;
    if (!st[seg].active) return;   // stopped: nothing reads the partials
    const double wmu_d = op.wmu[seg];
    const float wmu = (float)wmu_d;
    const int i = op.srow[sl * 64 + lane];
    const bool row = i < op.nrow_valid;
    // this row's r and diagonal do not depend on the product: loaded first
    const float2 rv = row ? R[i] : f2(0.f, 0.f);
    const double kd = row ? op.Kd[i] : 1.0, md = row ? op.Md[i] : 0.0;
    float2 ak = f2(0.f, 0.f), am = f2(0.f, 0.f);
    const int base = op.sp[sl], wd = op.sw[sl];
    int32_t cj[U];
    float kv[U], mv[U];
    auto fetch = [&](int k, int32_t* c, float* kk, float* mm) {
#pragma unroll
        for (int q = 0; q < U; ++q) {
            if (k + q < wd) {
                const int e = base + (k + q) * 64 + lane;
                c[q] = op.scol[e];
                kk[q] = op.sK[e];
                mm[q] = op.sM[e];
            } else {
                c[q] = row ? i : 0;
                kk[q] = 0.f;
                mm[q] = 0.f;
            }
        }
    };
    fetch(0, cj, kv, mv);
    for (int k = 0; k < wd; k += U) {
        float2 xv[U];
#pragma unroll
        for (int q = 0; q < U; ++q) xv[q] = X[cj[q]];
        int32_t cn[U];
        float kn[U], mn[U];
        if (k + U < wd) fetch(k + U, cn, kn, mn);
#pragma unroll
        for (int q = 0; q < U; ++q) {
            ak.x += kv[q] * xv[q].x; ak.y += kv[q] * xv[q].y;
            am.x += mv[q] * xv[q].x; am.y += mv[q] * xv[q].y;
        }
        if (k + U < wd) {
#pragma unroll
            for (int q = 0; q < U; ++q) { cj[q] = cn[q]; kv[q] = kn[q]; mv[q] = mn[q]; }
        }
    }
    double2 pq = make_double2(0.0, 0.0), qzr = pq, qzq = pq;
    if (row) {
        float2 y;
        y.x = ak.x + wmu * am.y;   // K x - i wmu M x
        y.y = ak.y - wmu * am.x;
        const float2 xo = X[i];
        const float2 zr = jacobi_z(rv, kd, md, wmu_d), zq = jacobi_z(y, kd, md, wmu_d);
        pq.x = (double)xo.x * y.x - (double)xo.y * y.y;
        pq.y = (double)xo.x * y.y + (double)xo.y * y.x;
        qzr.x = (double)y.x * zr.x - (double)y.y * zr.y;
        qzr.y = (double)y.x * zr.y + (double)y.y * zr.x;
        qzq.x = (double)y.x * zq.x - (double)y.y * zq.y;
        qzq.y = (double)y.x * zq.y + (double)y.y * zq.x;
        Y[i] = y;
    }
    const double s0 = wave_sum(pq.x), s1 = wave_sum(pq.y), s2 = wave_sum(qzr.x), s3 = wave_sum(qzr.y),
                 s4 = wave_sum(qzq.x), s5 = wave_sum(qzq.y);
    if (lane == 0) {
        red[wave][0] = make_double2(s0, s1);
        red[wave][1] = make_double2(s2, s3);
        red[wave][2] = make_double2(s4, s5);
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const int u = threadIdx.x;
        partial[(size_t)u * op.ntiles + tile] = cadd(cadd(red[0][u], red[1][u]), cadd(red[2][u], red[3][u]));
    }
}

// One block per mesh: fixed-order sums over the mesh's tiles of the
// product's three partials and the previous step's two, then the scalar step.
__global__ void __launch_bounds__(1024)
k_red_seg(Op op, ColState* __restrict__ st, const double2* __restrict__ ps, const double2* __restrict__ pg,
          const double2* __restrict__ pr) {
    __shared__ double2 red[16][5];
    __shared__ double2 tot[5];
    __shared__ ColState s_in;
    const int seg = blockIdx.x;
    if (!st[seg].active) return;   // the same in every thread
    // the state is copied to LDS first, so its load overlaps the sums
    if (threadIdx.x < sizeof(ColState) / 8)
        reinterpret_cast<double*>(&s_in)[threadIdx.x] = reinterpret_cast<const double*>(st + seg)[threadIdx.x];
    const int t0 = op.seg_tile[seg], t1 = op.seg_tile[seg + 1];
    double2 v[5];
#pragma unroll
    for (int j = 0; j < 5; ++j) v[j] = make_double2(0.0, 0.0);
    // four tiles per thread in flight
    for (int e0 = t0 + (int)threadIdx.x; e0 < t1; e0 += 4 * 1024) {
        double2 a[4][5];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = e0 + u * 1024;
            const bool ok = e < t1;
#pragma unroll
            for (int j = 0; j < 3; ++j) a[u][j] = ok ? ps[(size_t)j * op.ntiles + e] : make_double2(0.0, 0.0);
            a[u][3] = ok ? pg[e] : make_double2(0.0, 0.0);
            a[u][4] = ok ? pr[e] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int j = 0; j < 5; ++j) v[j] = cadd(v[j], a[u][j]);
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        const double sx = wave_sum(v[j].x), sy = wave_sum(v[j].y);
        if (lane == 0) red[wave][j] = make_double2(sx, sy);
    }
    __syncthreads();
    if (threadIdx.x < 5) {   // one sum per thread, the waves in order
        const int j = threadIdx.x;
        double2 a = red[0][j];
        for (int k = 1; k < 16; ++k) a = cadd(a, red[k][j]);
        tot[j] = a;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    ColState S = s_in;
    fused_scalars(S, tot);
    st[seg] = S;
}

// The row update of the fused step over one tile per block (the mesh's
// scalars from the state), with the tile's partials of the new r^T z and
// |r|^2 into go, ro.
__global__ void __launch_bounds__(256)
k_step_seg(Op op, const ColState* __restrict__ st, float2* __restrict__ R, const float2* __restrict__ Q,
           float2* __restrict__ P, float2* __restrict__ Xi, double2* __restrict__ go, double2* __restrict__ ro) {
    __shared__ double2 ra[256], rb[256];
    const int tile = tile_of(op, blockIdx.x);
    const int seg = op.tile_seg ? op.tile_seg[tile] : 0;
    const int i = tile * kTR + (int)threadIdx.x;
    const int ic = min(i, op.nrow_valid - 1);   // in range; the duplicate is not stored
    const float2 q = Q[ic], r = R[ic], x = Xi[ic], p = P[ic];
    const double kd = op.Kd[ic], md = op.Md[ic];
    const int active = st[seg].active;
    const double2 alpha = st[seg].alpha, beta = st[seg].beta;
    double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
    if (active && i < op.nrow_valid) {
        const float ax = (float)alpha.x, ay = (float)alpha.y, bx = (float)beta.x, by = (float)beta.y;
        float2 rr = r;
        rr.x -= ax * q.x - ay * q.y;
        rr.y -= ax * q.y + ay * q.x;
        const float2 z = jacobi_z(rr, kd, md, op.wmu[seg]);
        R[i] = rr;
        Xi[i] = f2(x.x + ax * p.x - ay * p.y, x.y + ax * p.y + ay * p.x);
        P[i] = f2(z.x + bx * p.x - by * p.y, z.y + bx * p.y + by * p.x);
        a.x = (double)rr.x * z.x - (double)rr.y * z.y;
        a.y = (double)rr.x * z.y + (double)rr.y * z.x;
        b.x = (double)rr.x * rr.x + (double)rr.y * rr.y;
    }
    cp_sum2(a, b, 1, ra, rb);
    if (threadIdx.x == 0) {
        go[tile] = ra[0];
        ro[tile] = rb[0];
    }
}

// x64 += |r64| d for the columns still refining. d is the inner solve's
// iterate, or for SQMR (XQ not null) its smoothed iterate x_Q: as the
// five-kernel iteration leaves it (lag 0), or with its last step still to
// take, x_Q = (1 - c^2) x_Q + c^2 x (lag 1, Eisenstat's form).
__global__ void __launch_bounds__(256)
k_ir_update(Op op, int CP, const ColState* __restrict__ st, const float2* __restrict__ Xi,
            const float2* __restrict__ XQ, int lag, double2* __restrict__ X64) {
    const int tile = blockIdx.x, C = op.C;
    const int c = threadIdx.x % CP, slot = threadIdx.x / CP, RPB = 256 / CP;
    if (c >= C) return;
    const int seg = op.tile_seg ? op.tile_seg[tile] : 0;
    const ColState& S = st[seg * C + c];
    if (!S.outer) return;
    const bool smooth = XQ && S.sqmr && S.kin > 0;
    const float cq = (float)S.cq, cp = (float)(1.0 - S.cq);
    for (int r0 = 0; r0 < kTR; r0 += RPB) {
        const int i = tile * kTR + r0 + slot;
        if (i >= op.nrow_valid) break;
        const size_t o = (size_t)i * C + c;
        float2 d = Xi[o];
        if (smooth) {
            if (lag) {
                const float2 xq = S.kin > 1 ? XQ[o] : f2(0.f, 0.f);
                d = f2(cp * xq.x + cq * d.x, cp * xq.y + cq * d.y);
            } else {
                d = XQ[o];
            }
        }
        double2 x = X64[o];
        x.x += S.scale * (double)d.x;
        x.y += S.scale * (double)d.y;
        X64[o] = x;
    }
}

// partial[tile][c].x = sum_i |B_ic|^2
__global__ void __launch_bounds__(256)
k_norm2(Op op, int CP, const double2* __restrict__ B, double2* __restrict__ p0) {
    __shared__ double2 ra[256];
    const int tile = blockIdx.x, C = op.C;
    const int c = threadIdx.x % CP, slot = threadIdx.x / CP, RPB = 256 / CP;
    double a = 0.0;
    if (c < C)
        for (int r0 = 0; r0 < kTR; r0 += RPB) {
            const int i = tile * kTR + r0 + slot;
            if (i >= op.nrow_valid) break;
            const double2 b = B[(size_t)i * C + c];
            a += b.x * b.x + b.y * b.y;
        }
    ra[threadIdx.x] = make_double2(a, 0.0);
    slot_tree(ra, CP, RPB);
    if ((int)threadIdx.x < C && (int)threadIdx.x < CP) p0[(size_t)tile * C + threadIdx.x] = ra[threadIdx.x];
}

// partials of w^H b and |w|^2 per (tile, column) for w = B - R (= A x)
__global__ void __launch_bounds__(256)
k_x0_dots(Op op, int CP, const double2* __restrict__ B, const double2* __restrict__ R, double2* __restrict__ p0,
          double2* __restrict__ p1) {
    __shared__ double2 ra[256], rb[256];
    const int tile = blockIdx.x, C = op.C;
    const int c = threadIdx.x % CP, slot = threadIdx.x / CP, RPB = 256 / CP;
    double2 a = make_double2(0.0, 0.0), b2 = make_double2(0.0, 0.0);
    if (c < C)
        for (int r0 = 0; r0 < kTR; r0 += RPB) {
            const int i = tile * kTR + r0 + slot;
            if (i >= op.nrow_valid) break;
            const size_t o = (size_t)i * C + c;
            const double2 bb = B[o];
            const double2 w = csub(bb, R[o]);
            a = cadd(a, cmulc(w, bb));
            b2.x += cabs2(w);
        }
    ra[threadIdx.x] = a;
    rb[threadIdx.x] = b2;
    slot_tree(ra, CP, RPB);
    slot_tree(rb, CP, RPB);
    if ((int)threadIdx.x < C && (int)threadIdx.x < CP) {
        p0[(size_t)tile * C + threadIdx.x] = ra[threadIdx.x];
        p1[(size_t)tile * C + threadIdx.x] = rb[threadIdx.x];
    }
}

// X = 0 in the (segment, column) pairs flagged
__global__ void __launch_bounds__(256)
k_zero_cols(Op op, int CP, const int* __restrict__ flags, double2* __restrict__ X) {
    const int tile = blockIdx.x, C = op.C;
    const int c = threadIdx.x % CP, slot = threadIdx.x / CP, RPB = 256 / CP;
    if (c >= C) return;
    const int seg = op.tile_seg ? op.tile_seg[tile] : 0;
    if (!flags[seg * C + c]) return;
    for (int r0 = 0; r0 < kTR; r0 += RPB) {
        const int i = tile * kTR + r0 + slot;
        if (i >= op.nrow_valid) break;
        X[(size_t)i * C + c] = make_double2(0.0, 0.0);
    }
}

// X *= alpha per column
__global__ void __launch_bounds__(256)
k_scale_cols(Op op, int CP, const ColState* __restrict__ st, double2* __restrict__ X) {
    const int tile = blockIdx.x, C = op.C;
    const int c = threadIdx.x % CP, slot = threadIdx.x / CP, RPB = 256 / CP;
    if (c >= C) return;
    const int seg = op.tile_seg ? op.tile_seg[tile] : 0;
    const double2 al = st[seg * C + c].alpha;
    for (int r0 = 0; r0 < kTR; r0 += RPB) {
        const int i = tile * kTR + r0 + slot;
        if (i >= op.nrow_valid) break;
        const size_t o = (size_t)i * C + c;
        X[o] = cmul(al, X[o]);
    }
}

__global__ void k_fill_f2(size_t n, float2* __restrict__ a) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) a[i] = make_float2(0.f, 0.f);
}

__global__ void k_fill_z(size_t n, double2* __restrict__ a) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) a[i] = make_double2(0.0, 0.0);
}

// dst[c][i] = src[i][c] (row-major block -> per-column vectors), rows [r0, r0+nr)
__global__ void k_cols_out(int nr, int C, size_t r0, const double2* __restrict__ src,
                           double2* __restrict__ dst, size_t ldd) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (size_t)nr * C) return;
    const size_t i = e / C, c = e % C;
    dst[c * ldd + i] = src[(r0 + i) * C + c];
}

__global__ void k_cols_in(int nr, int C, size_t r0, const double2* __restrict__ src, size_t lds,
                          double2* __restrict__ dst) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (size_t)nr * C) return;
    const size_t i = e / C, c = e % C;
    dst[(r0 + i) * C + c] = src[c * lds + i];
}

__global__ void k_init_state(ColState* st, int nsc, double inner_rtol, int sqmr) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nsc) return;
    ColState S;
    S.rho = S.alpha = S.beta = make_double2(0.0, 0.0);
    S.rn2 = 0.0;
    S.rn2_0 = 1.0;
    S.rn2_best = 0.0;
    S.scale = 0.0;
    S.bnorm = 0.0;
    S.rnorm64 = 0.0;
    S.tol_abs = 0.0;
    S.inner_tol2 = inner_rtol * inner_rtol;
    S.inner_rtol = inner_rtol;
    S.active = 0;
    S.outer = 1;
    S.breakdown = 0;
    S.iters = 0;
    S.kin = 0;
    S.stepped = 0;
    S.k_best = 0;
    S.stalled = 0;
    S.tau2 = 0.0;
    S.cq = 0.0;
    S.tmark = 0.0;
    S.sqmr = sqmr;
    st[k] = S;
}

// every column live (for the autotuner's timing launches)
__global__ void k_set_live(ColState* st, int nsc) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nsc) return;
    st[k].active = 1;
    st[k].outer = 1;
    st[k].kin = 0;
    st[k].beta = make_double2(0.0, 0.0);
    st[k].rho = make_double2(1.0, 0.0);
}

__global__ void k_set_tol(ColState* st, int nsc, double rtol) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nsc) return;
    st[k].tol_abs = rtol * st[k].bnorm;
    st[k].outer = st[k].bnorm > 0.0 && isfinite(st[k].bnorm);
}

// Builders of the concatenated (block-diagonal) operator of several meshes.
__global__ void k_cat_rows(int n, int32_t nnz_off, int row_off, const int32_t* __restrict__ rp,
                           int32_t* __restrict__ rp_cat) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i <= n) rp_cat[row_off + i] = rp[i] + nnz_off;
}
__global__ void k_fill_rp(int n, int32_t v, int32_t* __restrict__ a) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) a[i] = v;
}
__global__ void k_cat_cols(int64_t nnz, int row_off, const int32_t* __restrict__ col,
                           const double* __restrict__ K, const double* __restrict__ M,
                           int32_t* __restrict__ col_cat, double* __restrict__ K64,
                           double* __restrict__ M64, float* __restrict__ K32, float* __restrict__ M32) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= nnz) return;
    col_cat[k] = col[k] + row_off;
    K64[k] = K[k];
    M64[k] = M[k];
    K32[k] = (float)K[k];
    M32[k] = (float)M[k];
}
__global__ void k_fill_d(int n, double v, double* __restrict__ a) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) a[i] = v;
}

// Sliced-ELLPACK builders: the order of the rows inside each 256-row tile
// (by length, longest first, ties by index; rows past the last matrix row
// last), the width (longest row) of every 64-row slice, then the
// column-major fill of every slice (padding: zero values pointing at the row
// itself, or at row 0 for a lane past the last matrix row).
__global__ void __launch_bounds__(256)
k_sell_rows(int nrow_valid, const int32_t* __restrict__ rp, int32_t* __restrict__ row) {
    __shared__ int len[256];
    const int t = threadIdx.x, i = blockIdx.x * 256 + t;
    const int mine = i < nrow_valid ? rp[i + 1] - rp[i] : -1;
    len[t] = mine;
    __syncthreads();
    int rank = 0;
    for (int j = 0; j < 256; ++j) rank += (len[j] > mine) || (len[j] == mine && j < t);
    row[blockIdx.x * 256 + rank] = i;
}

__global__ void k_sell_width(int nsl, int nrow_valid, const int32_t* __restrict__ rp, const int32_t* __restrict__ row,
                             int32_t* __restrict__ w) {
    const int sl = blockIdx.x * blockDim.x + threadIdx.x;
    if (sl >= nsl) return;
    int m = 0;
    for (int l = 0; l < 64; ++l) {
        const int i = row[sl * 64 + l];
        if (i < nrow_valid) m = max(m, rp[i + 1] - rp[i]);
    }
    w[sl] = m;
}

__global__ void k_sell_fill(int nsl, int nrow_valid, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                            const float* __restrict__ K, const float* __restrict__ M, const int32_t* __restrict__ ptr,
                            const int32_t* __restrict__ w, const int32_t* __restrict__ row, int32_t* __restrict__ scol,
                            float* __restrict__ sK, float* __restrict__ sM, int values_only) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int sl = t >> 6, l = t & 63;
    if (sl >= nsl) return;
    const int i = row[sl * 64 + l];
    const int b = i < nrow_valid ? rp[i] : 0;
    const int len = i < nrow_valid ? rp[i + 1] - b : 0;
    const int wd = w[sl];
    for (int k = 0; k < wd; ++k) {
        const size_t e = (size_t)ptr[sl] + (size_t)k * 64 + l;
        if (k < len) {
            if (!values_only) scol[e] = col[b + k];
            sK[e] = K[b + k];
            sM[e] = M[b + k];
        } else {
            if (!values_only) scol[e] = i < nrow_valid ? i : 0;
            sK[e] = 0.f;
            sM[e] = 0.f;
        }
    }
}

}  // namespace

// ---------------------------------------------------------------- host side

struct SpmmChoice {
    int kind = 0;   // 0 = column lanes, 1 = nonzero lanes, 2 = sliced ELLPACK
    int a = 8, b = 1;   // (LPR, CPL), (G, CM) or (CM, U)
    float ms = 0.f;
};

struct SpmmTuned {
    SpmmChoice best;   // fastest complex64 shape
    SpmmChoice csr;    // fastest CSR shape (the double-precision residual uses it)
};

struct BlockWork {
    size_t cap_rows = 0;
    int cap_C = 0, cap_nsc = 0, cap_tiles = 0;
    double2 *X64 = nullptr, *R64 = nullptr, *B64 = nullptr;
    float2 *Xi = nullptr, *R = nullptr, *Z = nullptr, *P = nullptr, *Q = nullptr;
    float2* Dinv = nullptr;    // complex64 D^-1 of a single-column solve
    int p0_slots = 0;          // SpMM partial slots per tile that p0 holds
    size_t dinv_rows = 0;
    double2 *p0 = nullptr, *p1 = nullptr, *p2 = nullptr;
    double2* pe = nullptr;     // partials of the Eisenstat L pass, one slot per sweep block
    size_t pe_cap = 0;
    float2* XQ = nullptr;      // SQMR: the smoothed iterate of each column's inner solve
    size_t xq_cap = 0;
    ColState* st = nullptr;
    ColState* st2 = nullptr;   // second state slot of the in-consumer reductions
    ColState* st_h = nullptr;
    ColState* st_h2 = nullptr;             // second host snapshot of the state (overlapped checks)
    ColState* snap_ring = nullptr;         // [kSnapRing] host slots the fused step writes
    int* gcount = nullptr;                 // groups completed by the fused step (device)
    hipEvent_t snap_ev[2] = {nullptr, nullptr};
    int* tmap = nullptr;       // launched tiles of a compacted uneven batch
    int* flags = nullptr;      // [nsc] per-column flags (rejected initial guesses)
    double* wmu = nullptr;
    int* seg_tile = nullptr;
    int* tile_seg = nullptr;
    // concatenated operator of an uneven batch
    int32_t *rp = nullptr, *col = nullptr;
    double *K64 = nullptr, *M64 = nullptr, *Kd = nullptr, *Md = nullptr;
    float *K32 = nullptr, *M32 = nullptr;
    Sell cat_sell;
    size_t cat_rows = 0, cat_nnz = 0;
    std::map<std::tuple<int, int64_t, int>, SpmmTuned> tuned;   // (n, nnz, C) -> choices
    // graphs[k]: k + 1 iteration groups (captured when first needed)
    hipGraphExec_t graphs[kMaxGroups] = {};
    hipStream_t graph_stream = nullptr;
    std::vector<char> graph_sig;   // bytes of every argument baked into the graphs
    ~BlockWork() { release(); }
    void release_graph() {
        for (auto& g : graphs) {
            if (g) (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
        graph_sig.clear();
    }
    void release() {
        release_graph();
        if (graph_stream) (void)hipStreamDestroy(graph_stream);
        graph_stream = nullptr;
        dfree(X64); dfree(R64); dfree(B64); dfree(Xi); dfree(R); dfree(Z); dfree(P); dfree(Q);
        dfree(Dinv);
        dinv_rows = 0;
        dfree(p0); dfree(p1); dfree(p2); dfree(st); dfree(st2); dfree(tmap); dfree(flags); dfree(wmu);
        dfree(pe);
        pe_cap = 0;
        dfree(XQ);
        xq_cap = 0;
        dfree(seg_tile); dfree(tile_seg);
        dfree(rp); dfree(col); dfree(K64); dfree(M64); dfree(Kd); dfree(Md); dfree(K32); dfree(M32);
        cat_sell.release();
        if (st_h) (void)hipHostFree(st_h);
        st_h = nullptr;
        if (st_h2) (void)hipHostFree(st_h2);
        st_h2 = nullptr;
        if (snap_ring) (void)hipHostFree(snap_ring);
        snap_ring = nullptr;
        dfree(gcount);
        for (auto& e : snap_ev) {
            if (e) (void)hipEventDestroy(e);
            e = nullptr;
        }
        cap_rows = 0; cap_C = cap_nsc = cap_tiles = 0;
        cat_rows = cat_nnz = 0;
    }
};

void release_block_work(BlockWork*& w) {
    delete w;
    w = nullptr;
}

// (Re)build the sliced-ELLPACK copy of a complex64 operator of nrows rows
// (a multiple of the 256-row tile; rows from nrow_valid on are empty). The
// pattern is kept when `pattern` is false and the slice count is unchanged;
// the values are always refreshed.
int build_sell(Sell& S, int nrows, int nrow_valid, const int32_t* rp, const int32_t* col, const float* K,
               const float* M, bool pattern, hipStream_t s) {
    if (nrows % kTR != 0 || nrow_valid > nrows) {
        set_error("sliced ELLPACK: the rows must fill whole tiles");
        return PETGEM_INVALID_ARG;
    }
    const int nsl = nrows / 64;
    if (pattern || S.nsl != nsl || !S.ptr) {
        S.release();
        PG_TRY(dalloc(&S.ptr, (size_t)nsl + 1));
        PG_TRY(dalloc(&S.w, (size_t)nsl));
        PG_TRY(dalloc(&S.row, (size_t)nrows));
        hipLaunchKernelGGL(k_sell_rows, dim3(nrows / kTR), dim3(256), 0, s, nrow_valid, rp, S.row);
        hipLaunchKernelGGL(k_sell_width, dim3(ceil_div(nsl, 256)), dim3(256), 0, s, nsl, nrow_valid, rp, S.row, S.w);
        std::vector<int32_t> w(nsl), ptr(nsl + 1);
        PG_HIP(hipMemcpyAsync(w.data(), S.w, sizeof(int32_t) * nsl, hipMemcpyDeviceToHost, s));
        PG_HIP(hipStreamSynchronize(s));
        int64_t tot = 0;
        for (int k = 0; k < nsl; ++k) {
            ptr[k] = (int32_t)tot;
            tot += (int64_t)w[k] * 64;
            if (tot >= (int64_t(1) << 31)) {
                set_error("operator too large for 32-bit sliced-ELLPACK offsets");
                return PETGEM_INVALID_ARG;
            }
        }
        ptr[nsl] = (int32_t)tot;
        PG_HIP(hipMemcpyAsync(S.ptr, ptr.data(), sizeof(int32_t) * (nsl + 1), hipMemcpyHostToDevice, s));
        PG_TRY(dalloc(&S.col, (size_t)std::max<int64_t>(tot, 1)));
        PG_TRY(dalloc(&S.K, (size_t)std::max<int64_t>(tot, 1)));
        PG_TRY(dalloc(&S.M, (size_t)std::max<int64_t>(tot, 1)));
        S.nsl = nsl;
        S.elems = tot;
        hipLaunchKernelGGL(k_sell_fill, dim3(ceil_div((size_t)nsl * 64, 256)), dim3(256), 0, s, nsl, nrow_valid, rp,
                           col, K, M, S.ptr, S.w, S.row, S.col, S.K, S.M, 0);
        // the host vectors above must outlive the copy
        PG_HIP(hipStreamSynchronize(s));
    } else {
        hipLaunchKernelGGL(k_sell_fill, dim3(ceil_div((size_t)nsl * 64, 256)), dim3(256), 0, s, nsl, nrow_valid, rp,
                           col, K, M, S.ptr, S.w, S.row, S.col, S.K, S.M, 1);
    }
    PG_HIP(hipGetLastError());
    S.values = true;
    return PETGEM_OK;
}

// The multicolour split of the operator for SSOR (host build of the pattern
// on first use; values gathered on the GPU after every change of K32, Ms32).
// Colouring: the DOFs in the order of their global node pairs (lo, hi) (a
// numbering-free order), each taking the smallest colour none of its matrix
// neighbours already has.
int ensure_ssor(petgem_system* sys, hipStream_t s) {
    PG_TRY(ensure_fp32(sys, s));
    Ssor& Q = sys->ssor32;
    const int n = sys->n_dof;
    if (Q.nc == 0) {
        std::vector<int32_t> col((size_t)sys->nnz);
        PG_HIP(hipMemcpyAsync(col.data(), sys->col, sizeof(int32_t) * (size_t)sys->nnz, hipMemcpyDeviceToHost, s));
        PG_HIP(hipStreamSynchronize(s));
        const std::vector<int32_t>& rp = sys->row_ptr_h;
        std::vector<int32_t> order(n);
        for (int i = 0; i < n; ++i) order[i] = i;
        const int32_t* dn = sys->dof_nodes_h.data();
        std::sort(order.begin(), order.end(), [dn](int32_t a, int32_t b) {
            return dn[2 * a] != dn[2 * b] ? dn[2 * a] < dn[2 * b] : dn[2 * a + 1] < dn[2 * b + 1];
        });
        std::vector<int32_t> color(n, -1);
        std::vector<int32_t> seen;   // seen[c] == row: colour c taken by a neighbour of row
        int nc = 0;
        for (int32_t i : order) {
            for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
                const int32_t c = color[col[k]];
                if (c >= 0) seen[c] = i;
            }
            int32_t c = 0;
            while (c < nc && seen[c] == i) ++c;
            if (c == nc) { ++nc; seen.push_back(-1); }
            color[i] = c;
        }
        // rows listed colour by colour, in DOF order within a colour
        std::vector<int32_t> cptr(nc + 1, 0), row(n);
        for (int i = 0; i < n; ++i) ++cptr[color[i] + 1];
        for (int c = 0; c < nc; ++c) cptr[c + 1] += cptr[c];
        {
            std::vector<int32_t> fill(cptr.begin(), cptr.end() - 1);
            for (int i = 0; i < n; ++i) row[fill[color[i]]++] = i;
        }
        std::vector<int32_t> lrp(n + 1, 0), urp(n + 1, 0), lcol, lpos, ucol, upos;
        lcol.reserve((size_t)sys->nnz / 2); lpos.reserve((size_t)sys->nnz / 2);
        ucol.reserve((size_t)sys->nnz / 2); upos.reserve((size_t)sys->nnz / 2);
        for (int p = 0; p < n; ++p) {
            const int32_t i = row[p];
            for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
                const int32_t j = col[k];
                if (color[j] < color[i]) { lcol.push_back(j); lpos.push_back(k); }
                else if (color[j] > color[i]) { ucol.push_back(j); upos.push_back(k); }
                else if (j != i) {
                    set_error("SSOR colouring: two coupled unknowns share a colour");
                    return PETGEM_HIP_ERROR;
                }
            }
            lrp[p + 1] = (int32_t)lcol.size();
            urp[p + 1] = (int32_t)ucol.size();
        }
        Q.nl = (int64_t)lcol.size();
        Q.nu = (int64_t)ucol.size();
        PG_TRY(dalloc(&Q.row, (size_t)n));
        PG_TRY(dalloc(&Q.lrp, (size_t)n + 1));
        PG_TRY(dalloc(&Q.urp, (size_t)n + 1));
        PG_TRY(dalloc(&Q.lcol, (size_t)std::max<int64_t>(Q.nl, 1)));
        PG_TRY(dalloc(&Q.lpos, (size_t)std::max<int64_t>(Q.nl, 1)));
        PG_TRY(dalloc(&Q.ucol, (size_t)std::max<int64_t>(Q.nu, 1)));
        PG_TRY(dalloc(&Q.upos, (size_t)std::max<int64_t>(Q.nu, 1)));
        PG_TRY(dalloc(&Q.lK, (size_t)std::max<int64_t>(Q.nl, 1)));
        PG_TRY(dalloc(&Q.lM, (size_t)std::max<int64_t>(Q.nl, 1)));
        PG_TRY(dalloc(&Q.uK, (size_t)std::max<int64_t>(Q.nu, 1)));
        PG_TRY(dalloc(&Q.uM, (size_t)std::max<int64_t>(Q.nu, 1)));
        PG_TRY(dalloc(&Q.dg, (size_t)n));
        PG_HIP(hipMemcpyAsync(Q.row, row.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
        PG_HIP(hipMemcpyAsync(Q.lrp, lrp.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, s));
        PG_HIP(hipMemcpyAsync(Q.urp, urp.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, s));
        PG_HIP(hipMemcpyAsync(Q.lcol, lcol.data(), sizeof(int32_t) * lcol.size(), hipMemcpyHostToDevice, s));
        PG_HIP(hipMemcpyAsync(Q.lpos, lpos.data(), sizeof(int32_t) * lpos.size(), hipMemcpyHostToDevice, s));
        PG_HIP(hipMemcpyAsync(Q.ucol, ucol.data(), sizeof(int32_t) * ucol.size(), hipMemcpyHostToDevice, s));
        PG_HIP(hipMemcpyAsync(Q.upos, upos.data(), sizeof(int32_t) * upos.size(), hipMemcpyHostToDevice, s));
        PG_HIP(hipStreamSynchronize(s));   // the host vectors die here
        Q.cptr = std::move(cptr);
        Q.color_h = std::move(color);
        Q.nc = nc;
        Q.values = false;
    }
    if (!Q.values) {
        if (Q.nl > 0)
            hipLaunchKernelGGL(k_ssor_vals, dim3(ceil_div(Q.nl, 256)), dim3(256), 0, s, Q.nl, Q.lpos, sys->K32,
                               sys->Ms32, Q.lK, Q.lM);
        if (Q.nu > 0)
            hipLaunchKernelGGL(k_ssor_vals, dim3(ceil_div(Q.nu, 256)), dim3(256), 0, s, Q.nu, Q.upos, sys->K32,
                               sys->Ms32, Q.uK, Q.uM);
        hipLaunchKernelGGL(k_ssor_dg, dim3(ceil_div(n, 256)), dim3(256), 0, s, n, (const int32_t*)Q.row,
                           (const double*)sys->Kd, (const double*)sys->Msd, Q.dg);
        PG_HIP(hipGetLastError());
        Q.values = true;
    }
    return PETGEM_OK;
}

namespace {

// One multicolour pass of the sweep kernels over op's columns: the L entries
// with the colours ascending, or the U entries descending; bwd picks the
// backward formula z -= omega s / d, else z = omega (r - s) / d (a solve
// with D~ + L, or with D~ + U on the U entries). st (or null) skips stopped
// columns.
void ssor_pass(const Ssor& Q, const Op& op, const ColState* st, const float2* R, float2* Z, float omega,
               bool upper, bool bwd, hipStream_t s) {
    const int C = op.C;
    SsorOp so{Q.row, upper ? Q.urp : Q.lrp, upper ? Q.ucol : Q.lcol, upper ? Q.uK : Q.lK, upper ? Q.uM : Q.lM, Q.dg};
    for (int k = 0; k < Q.nc; ++k) {
        const int c = upper ? Q.nc - 1 - k : k;
        const int p0 = Q.cptr[c], p1 = Q.cptr[c + 1];
        if (p1 <= p0) continue;
#define PG_SN(G, CM) { const dim3 gr(ceil_div(p1 - p0, 256 / G)); \
        if (bwd) hipLaunchKernelGGL((k_ssor_n<G, CM, true>), gr, dim3(256), 0, s, op, so, p0, p1, st, R, Z, omega); \
        else hipLaunchKernelGGL((k_ssor_n<G, CM, false>), gr, dim3(256), 0, s, op, so, p0, p1, st, R, Z, omega); }
#define PG_SC(L, P) { const dim3 gr(ceil_div(p1 - p0, 256 / L)); \
        if (bwd) hipLaunchKernelGGL((k_ssor_c<L, P, true>), gr, dim3(256), 0, s, op, so, p0, p1, st, R, Z, omega); \
        else hipLaunchKernelGGL((k_ssor_c<L, P, false>), gr, dim3(256), 0, s, op, so, p0, p1, st, R, Z, omega); }
        if (C == 1) PG_SN(8, 1)
        else if (C == 2) PG_SN(8, 2)
        else if (C <= 4) PG_SN(8, 4)
        else if (C <= 8) PG_SC(8, 1)
        else if (C <= 16) PG_SC(16, 1)
        else if (C <= 32) PG_SC(32, 1)
        else if (C <= 64) PG_SC(64, 1)
        else if (C <= 128) PG_SC(64, 2)
        else PG_SC(64, 4)
#undef PG_SN
#undef PG_SC
    }
}

// z = M^-1 r by the two multicolour sweeps (Z in place; R read by the
// forward sweep).
void ssor_sweeps(const Ssor& Q, const Op& op, const ColState* st, const float2* R, float2* Z, float omega,
                 hipStream_t s) {
    ssor_pass(Q, op, st, R, Z, omega, false, false, s);
    ssor_pass(Q, op, st, R, Z, omega, true, true, s);
}

// Lanes per row of the many-column sweep kernels (C > 4).
int eis_lpr(int C) { return C <= 8 ? 8 : C <= 16 ? 16 : C <= 32 ? 32 : 64; }

// Blocks of one colour of the Eisenstat L pass: each strides over the
// colour's rows, at most kEisBlocks of them (the partial slots stay few).
constexpr int kEisBlocks = 2048;
int eis_blocks(int rows, int C) { return std::min(ceil_div(rows, 256 / eis_lpr(C)), kEisBlocks); }

// Blocks of one Eisenstat L pass (its partial slots).
int eis_slots(const Ssor& Q, int C) {
    int n = 0;
    for (int c = 0; c < Q.nc; ++c) n += eis_blocks(Q.cptr[c + 1] - Q.cptr[c], C);
    return n;
}

template <typename K, typename... Args>
void launch_timed(K kernel, dim3 grid, hipStream_t s, hipEvent_t e0, hipEvent_t e1, Args... args);

// The Eisenstat U pass with the direction update (k_ssor_eis_u), colours
// descending. evs (or null): every launch timestamps its start and end into
// a new pair of events appended there (the profile of the solve; this pass
// has the largest total time of the iteration).
void eis_upass(const Ssor& Q, const Op& op, const ColState* st, const float2* R, float2* P, float2* T, float omega,
               hipStream_t s, std::vector<hipEvent_t>* evs) {
    const int C = op.C;
    const SsorOp so{Q.row, Q.urp, Q.ucol, Q.uK, Q.uM, Q.dg};
    for (int k = 0; k < Q.nc; ++k) {
        const int c = Q.nc - 1 - k;
        const int p0 = Q.cptr[c], p1 = Q.cptr[c + 1];
        if (p1 <= p0) continue;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (evs) {
            (void)hipEventCreate(&e0);
            (void)hipEventCreate(&e1);
            evs->push_back(e0);
            evs->push_back(e1);
        }
#define PG_SU(L, PP) launch_timed((k_ssor_eis_u<L, PP>), dim3(ceil_div(p1 - p0, 256 / L)), s, e0, e1, op, so, \
                                  p0, p1, st, R, P, T, omega);
        if (C <= 8) PG_SU(8, 1)
        else if (C <= 16) PG_SU(16, 1)
        else if (C <= 32) PG_SU(32, 1)
        else if (C <= 64) PG_SU(64, 1)
        else if (C <= 128) PG_SU(64, 2)
        else PG_SU(64, 4)
#undef PG_SU
    }
}

// The Eisenstat L pass (k_ssor_eis), colours ascending, block partials in
// launch order, column c's from part + c * cs.
void eis_lpass(const Ssor& Q, const Op& op, const ColState* st, const float2* P, const float2* T, float2* Y,
               float omega, double2* part, int64_t cs, hipStream_t s) {
    const int C = op.C;
    const SsorOp so{Q.row, Q.lrp, Q.lcol, Q.lK, Q.lM, Q.dg};
    int base = 0;
    for (int c = 0; c < Q.nc; ++c) {
        const int p0 = Q.cptr[c], p1 = Q.cptr[c + 1];
        if (p1 <= p0) continue;
#define PG_SE(L, PP) { const int nb = eis_blocks(p1 - p0, C); \
        hipLaunchKernelGGL((k_ssor_eis<L, PP>), dim3(nb), dim3(256), 0, s, op, so, p0, p1, st, P, T, Y, omega, \
                           part, base, cs); \
        base += nb; }
        if (C <= 8) PG_SE(8, 1)
        else if (C <= 16) PG_SE(16, 1)
        else if (C <= 32) PG_SE(32, 1)
        else if (C <= 64) PG_SE(64, 1)
        else if (C <= 128) PG_SE(64, 2)
        else PG_SE(64, 4)
#undef PG_SE
    }
}

}  // namespace

int ssor_apply1(petgem_system* sys, double freq, double omega, const float2* r, float2* z, hipStream_t s) {
    PG_TRY(ensure_ssor(sys, s));
    double* wmu = nullptr;
    PG_TRY(dalloc(&wmu, 1));
    const double w = 2.0 * kPi * freq * kMu0;
    PG_HIP(hipMemcpyAsync(wmu, &w, sizeof(double), hipMemcpyHostToDevice, s));
    Op op{};
    op.n = sys->n_dof;
    op.C = 1;
    op.ntiles = ceil_div(sys->n_dof, kTR);
    op.nlaunch = op.ntiles;
    op.nseg = 1;
    op.Kd = sys->Kd;
    op.Md = sys->Msd;
    op.wmu = wmu;
    op.nrow_valid = sys->n_dof;
    ssor_sweeps(sys->ssor32, op, nullptr, r, z, (float)omega, s);
    PG_HIP(hipGetLastError());
    PG_HIP(hipStreamSynchronize(s));
    dfree(wmu);
    return PETGEM_OK;
}

namespace {

// Launch arguments of one SpMM (X, B, Y as described at the kernels; e0 / e1
// optional events the dispatch timestamps at the kernel's start and end).
struct SpmmArgs {
    const void* X;
    const void* B;
    void* Y;
    double2* part;
    hipEvent_t e0 = nullptr;
    hipEvent_t e1 = nullptr;
};

// launch through the timestamping dispatch only when events are given (plain
// launches are what the graphs capture)
template <typename K, typename... Args>
void launch_timed(K kernel, dim3 grid, hipStream_t s, hipEvent_t e0, hipEvent_t e1, Args... args) {
    if (e0)
        hipExtLaunchKernelGGL(kernel, grid, dim3(256), 0, s, e0, e1, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, dim3(256), 0, s, args...);
}

template <typename K, typename... Args>
void launch_timed_b(K kernel, dim3 grid, dim3 block, hipStream_t s, hipEvent_t e0, hipEvent_t e1, Args... args) {
    if (e0)
        hipExtLaunchKernelGGL(kernel, grid, block, 0, s, e0, e1, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
}

// nonzeros per trip of k_spmm_g: 20 (every row of the Kuhn meshes in one
// trip), fewer where the gathered values of a trip would need more than
// about 160 registers per lane
template <typename T, int CPL>
constexpr int spmm_g_nb() {
    constexpr int per = CPL * 2 * (int)sizeof(T) / 4;   // registers per gathered nonzero
    constexpr int nb = 160 / per;
    return nb > 20 ? 20 : (nb < 4 ? 4 : nb);
}

template <typename T, int A, int B, int EPI>
void spmm_thunk_g(Op op, const ColState* st, const SpmmArgs& g, hipStream_t s) {
    using T2 = typename V2<T>::t;
    launch_timed(k_spmm_g<T, A, B, spmm_g_nb<T, B>(), EPI>, dim3(op.nlaunch), s, g.e0, g.e1, op, st,
                 (const T2*)g.X, (const T2*)g.B, (T2*)g.Y, g.part);
}

template <typename T, int A, int B, int EPI, bool COLS>
void spmm_thunk(Op op, const ColState* st, const SpmmArgs& g, hipStream_t s) {
    using T2 = typename V2<T>::t;
    if constexpr (COLS)
        launch_timed(k_spmm_c<T, A, B, EPI>, dim3(op.nlaunch), s, g.e0, g.e1, op, st, (const T2*)g.X,
                     (const T2*)g.B, (T2*)g.Y, g.part);
    else
        launch_timed(k_spmm_n<T, A, B, EPI>, dim3(op.nlaunch * A), s, g.e0, g.e1, op, st, (const T2*)g.X,
                     (const T2*)g.B, (T2*)g.Y, g.part);
}

template <typename T, int EPI>
bool spmm_dispatch_(const SpmmChoice& ch, Op op, const ColState* st, const SpmmArgs& g, hipStream_t s) {
    if (ch.kind == 2) {
        if constexpr (sizeof(T) == 4 && EPI == 1) {
            if (!op.sp) return false;
#define PG_S(CM, U) if (ch.a == CM && ch.b == U) { \
            launch_timed(k_spmm_s<CM, U>, dim3(op.nlaunch), s, g.e0, g.e1, op, st, (const float2*)g.X, \
                         (float2*)g.Y, g.part); return true; }
            PG_S(1, 4) PG_S(1, 8) PG_S(2, 4) PG_S(2, 8) PG_S(4, 4)
#undef PG_S
        }
        return false;
    }
    if (ch.kind == 3) {
        if constexpr (sizeof(T) == 4 && EPI == 1) {
            if (!op.sp) return false;
#define PG_SP(CM, U) if (ch.a == CM && ch.b == U) { \
            launch_timed(k_spmm_sp<CM, U>, dim3(op.nlaunch), s, g.e0, g.e1, op, st, (const float2*)g.X, \
                         (float2*)g.Y, g.part); return true; }
            PG_SP(1, 4) PG_SP(1, 8) PG_SP(2, 4)
#undef PG_SP
        }
        return false;
    }
    if (ch.kind == 6) {
#define PG_G(L, P) if (ch.a == L && ch.b == P) { spmm_thunk_g<T, L, P, EPI>(op, st, g, s); return true; }
        PG_G(8, 1) PG_G(8, 2) PG_G(8, 4) PG_G(16, 1) PG_G(16, 2) PG_G(16, 3) PG_G(16, 4) PG_G(32, 1) PG_G(32, 2)
        PG_G(64, 1)
#undef PG_G
        return false;
    }
    if (ch.kind == 1) {
#define PG_N(G, CM) if (ch.a == G && ch.b == CM) { spmm_thunk<T, G, CM, EPI, false>(op, st, g, s); return true; }
        PG_N(4, 1) PG_N(8, 1) PG_N(16, 1) PG_N(4, 2) PG_N(8, 2) PG_N(16, 2) PG_N(4, 4) PG_N(8, 4) PG_N(16, 4)
#undef PG_N
    } else {
#define PG_C(L, P) if (ch.a == L && ch.b == P) { spmm_thunk<T, L, P, EPI, true>(op, st, g, s); return true; }
        PG_C(8, 1) PG_C(8, 2) PG_C(8, 4) PG_C(16, 1) PG_C(16, 2) PG_C(16, 3) PG_C(16, 4)
        PG_C(32, 1) PG_C(32, 2) PG_C(32, 3) PG_C(32, 4) PG_C(64, 1) PG_C(64, 2) PG_C(64, 3) PG_C(64, 4)
#undef PG_C
    }
    return false;
}

template <typename T, int EPI>
void spmm_dispatch(const SpmmChoice& ch, Op op, const ColState* st, const SpmmArgs& g, hipStream_t s) {
    if (!spmm_dispatch_<T, EPI>(ch, op, st, g, s)) abort();   // candidates() lists only instantiated shapes
}

// partial slots per tile of an SpMM shape
int spmm_slots(const SpmmChoice& ch) { return ch.kind == 1 ? ch.a : 1; }
// shapes on the CSR arrays, which also serve the double-precision residual
bool csr_kind(const SpmmChoice& ch) { return ch.kind == 0 || ch.kind == 1 || ch.kind == 6; }


std::vector<SpmmChoice> candidates(int C, bool sell) {
    std::vector<SpmmChoice> v;
    if (C <= 4) {
        const int cm = C <= 1 ? 1 : (C <= 2 ? 2 : 4);
        for (int g : {4, 8, 16}) v.push_back({1, g, cm});
        if (sell) {
            v.push_back({2, cm, 4});
            if (cm < 4) v.push_back({2, cm, 8});
            if (cm == 1) v.push_back({3, 1, 8});
            if (cm <= 2) v.push_back({3, cm, 4});
        }
    }
    if (C >= 4) {
        for (int l : {8, 16, 32, 64})
            for (int p : {1, 2, 3, 4}) {
                if (l == 8 && p == 3) continue;
                if (l * p < C) continue;
                if (l * p >= 2 * C && l > 8) continue;   // more than half the lanes idle
                v.push_back({0, l, p});
            }
        if (v.empty() || (C > 256)) v.push_back({0, 64, 4});
        // the same lane shapes with the row's entries spread over its lanes
        // (kind 6), up to 64 columns and 32 columns per lane group
        for (int l : {8, 16, 32, 64})
            for (int p : {1, 2, 3, 4}) {
                const bool inst = (l == 8 && p != 3) || (l == 16) || (l == 32 && p <= 2) || (l == 64 && p == 1);
                if (!inst || l * p < C || (l * p >= 2 * C && l > 8) || C > 64) continue;
                v.push_back({6, l, p});
            }
    }
    return v;
}

struct Timer {
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    double ms() const {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
};

int ensure_work(BlockWork*& w, size_t rows, int C, int nsc, int ntiles) {
    if (!w) w = new BlockWork();
    if (w->cap_rows >= rows && w->cap_C == C && w->cap_nsc >= nsc && w->cap_tiles >= ntiles) return PETGEM_OK;
    // keep the concatenated operator, reallocate the vectors
    w->release_graph();
    dfree(w->X64); dfree(w->R64); dfree(w->B64); dfree(w->Xi); dfree(w->R); dfree(w->Z); dfree(w->P);
    dfree(w->Q);
    dfree(w->p0); dfree(w->p1); dfree(w->p2); dfree(w->st); dfree(w->st2); dfree(w->tmap); dfree(w->flags); dfree(w->wmu); dfree(w->seg_tile); dfree(w->tile_seg);
    if (w->st_h) (void)hipHostFree(w->st_h);
    w->st_h = nullptr;
    if (w->st_h2) (void)hipHostFree(w->st_h2);
    w->st_h2 = nullptr;
    const size_t e = rows * (size_t)C;
    PG_TRY(dalloc(&w->X64, e));
    PG_TRY(dalloc(&w->R64, e));
    PG_TRY(dalloc(&w->B64, e));
    PG_TRY(dalloc(&w->Xi, e));
    PG_TRY(dalloc(&w->R, e));
    PG_TRY(dalloc(&w->Z, e));
    PG_TRY(dalloc(&w->P, e));
    PG_TRY(dalloc(&w->Q, e));
    // SpMM partial slots per tile: up to 16 for the nonzero-lane shapes (few
    // columns), one otherwise
    w->p0_slots = C <= 4 ? 16 : 1;
    PG_TRY(dalloc(&w->p0, (size_t)ntiles * C * w->p0_slots));
    // p1, p2: per-tile or per-block partials; the fused single-column step
    // keeps two halves of ceil(ntiles / kStepTiles) blocks each
    const size_t np12 = std::max((size_t)ntiles * C, 2 * (size_t)ceil_div(ntiles, kStepTiles));
    PG_TRY(dalloc(&w->p1, np12));
    PG_TRY(dalloc(&w->p2, np12));

    PG_TRY(dalloc(&w->st, (size_t)nsc));
    PG_TRY(dalloc(&w->st2, (size_t)nsc));
    PG_TRY(dalloc(&w->flags, (size_t)nsc));
    PG_TRY(dalloc(&w->wmu, (size_t)nsc));
    PG_TRY(dalloc(&w->seg_tile, (size_t)nsc + 1));
    PG_TRY(dalloc(&w->tile_seg, (size_t)ntiles));
    PG_HIP(hipHostMalloc(reinterpret_cast<void**>(&w->st_h), sizeof(ColState) * (size_t)nsc));
    PG_HIP(hipHostMalloc(reinterpret_cast<void**>(&w->st_h2), sizeof(ColState) * (size_t)nsc));
    for (auto& e : w->snap_ev)
        if (!e) PG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    w->cap_rows = rows;
    w->cap_C = C;
    w->cap_nsc = nsc;
    w->cap_tiles = ntiles;
    return PETGEM_OK;
}

int cp_of(int C) {
    int cp = 1;
    while (cp < C && cp < 256) cp <<= 1;
    return cp;
}

// Autotuner of the complex64 SpMM tile shape: every candidate (lanes per row x
// columns per lane, or lanes sharing a row's nonzeros) runs 3 times on this
// operator and block width; the fastest is kept per (rows, nnz, columns).
int tune_spmm(BlockWork* w, const Op& op, int64_t nnz, hipStream_t s, SpmmTuned& out, bool verbose) {
    auto key = std::make_tuple(op.n, nnz, op.C);
    auto it = w->tuned.find(key);
    if (it != w->tuned.end()) { out = it->second; return PETGEM_OK; }
    auto cands = candidates(op.C, op.sp != nullptr);
    // P (complex64, rows x C) gets finite values and every column is live
    // for the timing launches (the solve initialises both afterwards)
    const int nsc = op.nseg * op.C;
    hipLaunchKernelGGL(k_fill_f2, dim3(ceil_div((size_t)op.n * op.C, 256)), dim3(256), 0, s,
                       (size_t)op.n * op.C, w->P);
    hipLaunchKernelGGL(k_set_live, dim3(ceil_div(nsc, 64)), dim3(64), 0, s, w->st, nsc);
    static const char* kinds[7] = {"column lanes", "nonzero lanes", "sliced ELLPACK", "pipelined sliced ELLPACK",
                                   "fused", "fused per mesh", "column lanes, entries over the lanes"};
    hipEvent_t e0, e1;
    PG_HIP(hipEventCreate(&e0));
    PG_HIP(hipEventCreate(&e1));
    SpmmTuned best;
    best.best.ms = best.csr.ms = 1e30f;
    for (auto& c : cands) {
        if (spmm_slots(c) > w->p0_slots) continue;   // more partial slots than p0 holds
        const SpmmArgs g{w->P, nullptr, w->Q, w->p0};
        spmm_dispatch<float, 1>(c, op, w->st, g, s);   // warm-up
        PG_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < 3; ++r) spmm_dispatch<float, 1>(c, op, w->st, g, s);
        PG_HIP(hipEventRecord(e1, s));
        PG_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        PG_HIP(hipEventElapsedTime(&ms, e0, e1));
        c.ms = ms / 3.f;
        if (verbose) {
            fprintf(stderr, "[petgem] SpMM tuning: %s %d x %d: %.1f us\n", kinds[c.kind], c.a, c.b, 1e3 * c.ms);
            fflush(stderr);
        }
        if (c.ms < best.best.ms) best.best = c;
        if (csr_kind(c) && c.ms < best.csr.ms) best.csr = c;
    }
    // The double-precision residual of a few columns times the CSR shapes in
    // double (it reads X64 and B64 as they are and writes R64, all of which
    // the solve rewrites before use); more columns keep the complex64 order.
    if (op.C <= 4) {
        best.csr.ms = 1e30f;
        for (SpmmChoice c : cands) {
            if (!csr_kind(c) || spmm_slots(c) > w->p0_slots) continue;
            const SpmmArgs g{w->X64, w->B64, w->R64, w->p0};
            spmm_dispatch<double, 2>(c, op, w->st, g, s);   // warm-up
            PG_HIP(hipEventRecord(e0, s));
            for (int r = 0; r < 3; ++r) spmm_dispatch<double, 2>(c, op, w->st, g, s);
            PG_HIP(hipEventRecord(e1, s));
            PG_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            PG_HIP(hipEventElapsedTime(&ms, e0, e1));
            c.ms = ms / 3.f;
            if (verbose) {
                fprintf(stderr, "[petgem] SpMM tuning: double residual, %s %d x %d: %.1f us\n", kinds[c.kind], c.a,
                        c.b, 1e3 * c.ms);
                fflush(stderr);
            }
            if (c.ms < best.csr.ms) best.csr = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    w->tuned[key] = best;
    out = best;
    return PETGEM_OK;
}

// The driver shared by the multi-source and the uneven-batch solves.
// On entry B64 holds the right-hand sides, X64 the initial guesses (or zero).
// has_x0: which (segment, column) pairs came with an initial guess (null:
// all of them when have_x0); only those can be rejected.
int mrhs_solve(BlockWork* w, const Op& op, int64_t nnz, const petgem_opts& o, hipStream_t s,
               std::vector<petgem_stats*>& stv, bool have_x0, const std::vector<int>* seg_tile_h = nullptr,
               const std::vector<char>* has_x0 = nullptr, const Ssor* sq = nullptr) {
    const int C = op.C, nsc = op.nseg * C, CP = cp_of(C);
    // multicolour SSOR instead of Jacobi (one mesh): the five-kernel
    // iteration with the two sweeps and an r^T z pass between the r update
    // and the beta reduction
    const bool ssor = sq != nullptr;
    const float omega = (float)o.omega;
    // symmetric QMR: the same iteration with the smoothed iterate x_Q beside x
    const bool sqmr = o.method == PETGEM_SQMR;
    Timer t_all;
    SpmmTuned tu;
    PG_TRY(tune_spmm(w, op, nnz, s, tu, o.verbose != 0));
    // a caller-chosen fused step (kind 4: one column of one mesh, kind 5: one
    // column per mesh with a reduction block per mesh), with 4 or 8 slice
    // columns in flight; the other kernels keep the tuned shapes
    const int force_kind = o.spmm_shape / 10000;
    const bool force_fused = (force_kind == 4 || force_kind == 5) && o.spmm_shape % 10000 / 100 == 1 &&
                             (o.spmm_shape % 100 == 4 || o.spmm_shape % 100 == 8);
    if (force_fused && ssor) {
        set_error("the fused steps take the Jacobi preconditioner only");
        return PETGEM_INVALID_ARG;
    }
    if (force_fused && (C != 1 || op.sp == nullptr)) {
        set_error("spmm_shape " + std::to_string(o.spmm_shape) + " (a fused step) needs one column per mesh");
        return PETGEM_INVALID_ARG;
    }
    if (o.spmm_shape != 0 && !force_fused) {   // a caller-chosen shape instead of the tuned one
        bool found = false;
        for (const SpmmChoice& c : candidates(op.C, op.sp != nullptr))
            if (10000 * c.kind + 100 * c.a + c.b == o.spmm_shape) {
                tu.best = c;
                if (csr_kind(c)) tu.csr = c;
                found = true;
            }
        if (!found) {
            set_error("spmm_shape " + std::to_string(o.spmm_shape) + " is not a candidate for " +
                      std::to_string(op.C) + " columns");
            return PETGEM_INVALID_ARG;
        }
    }
    const SpmmChoice ch = tu.best, ch64 = tu.csr;
    const int ppS = spmm_slots(ch), pp64 = spmm_slots(ch64);
    if (ppS > w->p0_slots || pp64 > w->p0_slots) {
        set_error("SpMM shape " + std::to_string(10000 * ch.kind + 100 * ch.a + ch.b) + " needs " +
                  std::to_string(ppS) + " partial slots per tile; the work space holds " +
                  std::to_string(w->p0_slots));
        return PETGEM_INVALID_ARG;
    }
    // the reductions run inside the vector kernels for one mesh whose
    // partials are few enough for every block to sum
    const bool in_consumer = !ssor && op.nseg == 1 && (int64_t)op.ntiles * ppS * C <= kConsumerMax;
    const int nspb = ceil_div((int64_t)op.ntiles * 4, kSpbWaves);   // blocks (and partials) of the fused product
    const int nst = ceil_div(op.ntiles, kStepTiles);                // blocks of the fused step
    // One column of one mesh with a sliced-ELLPACK copy takes the fused step
    // (the product with its two extra partials, then one vector kernel) when
    // every step block can sum the product's partials, whichever product
    // shape the tuner timed fastest on its own: the step saves more than the
    // shapes differ (its own product is the pipelined one with 4 slice
    // columns in flight; 8 measured 2 % slower). The gate depends on the
    // fused kernels' own partial counts only, never on the tuned shape, so
    // the kernel path does not follow the tuner's timing noise. A
    // caller-chosen shape is honoured as given: shape 3 (or 4) runs fused,
    // the others not.
    const bool fused_fits = !ssor && op.nseg == 1 && C == 1 && op.sp != nullptr && nspb <= kConsumerMax;
    const bool fused = fused_fits && force_kind != 5 &&
                       (o.spmm_shape == 0 || force_kind == 4 ||
                        (ch.kind == 3 && ch.a == 1 && (ch.b == 4 || ch.b == 8)));
    const int fused_u = o.spmm_shape == 0 ? 4 : force_fused ? o.spmm_shape % 100 : ch.b;
    if (force_kind == 4 && !fused) {
        set_error("spmm_shape " + std::to_string(o.spmm_shape) + " (the fused single-column step) needs one mesh "
                  "of at most " + std::to_string(kConsumerMax) + " tiles");
        return PETGEM_INVALID_ARG;
    }
    // one column of one system: D^-1 once per solve in complex64 (an uneven
    // batch keeps the double-precision diagonal: its hardest models need a few
    // percent more iterations with the rounded D^-1)
    const float2* dinv = nullptr;
    if ((in_consumer && C == 1) || fused) {
        const size_t rows = (size_t)op.ntiles * kTR;
        if (w->dinv_rows < rows) {
            dfree(w->Dinv);
            w->dinv_rows = 0;
            PG_TRY(dalloc(&w->Dinv, rows));
            w->dinv_rows = rows;
        }
        hipLaunchKernelGGL(k_dinv, dim3(ceil_div(rows, 256)), dim3(256), 0, s, op, w->Dinv);
        PG_HIP(hipGetLastError());
        dinv = w->Dinv;
    }
    // SSOR with more than four columns: Eisenstat's form (no product with A
    // in the iteration); its L pass leaves one partial slot per block and
    // column, ntiles * ppE slots per column (the unused ones zero), and its
    // two reductions read their partials column by column (k_reduce_cm)
    const bool eis = ssor && C > 4;
    int ppE = 0, neis = 0;
    if (eis) {
        if (op.nseg != 1) {
            set_error("multicolour SSOR: one system only");
            return PETGEM_INVALID_ARG;
        }
        neis = eis_slots(*sq, C);
        ppE = ceil_div(eis_slots(*sq, C), op.ntiles);
        const size_t need = (size_t)op.ntiles * ppE * C;
        if (w->pe_cap < need) {
            dfree(w->pe);
            w->pe_cap = 0;
            PG_TRY(dalloc(&w->pe, need));
            w->pe_cap = need;
        }
        hipLaunchKernelGGL(k_fill_z, dim3(ceil_div(need, 256)), dim3(256), 0, s, need, w->pe);
        PG_HIP(hipGetLastError());
    }
    if (sqmr) {
        const size_t nxq = (size_t)op.n * C;
        if (w->xq_cap < nxq) {
            dfree(w->XQ);
            w->xq_cap = 0;
            PG_TRY(dalloc(&w->XQ, nxq));
            w->xq_cap = nxq;
        }
    }
    float2* const xq = sqmr ? w->XQ : nullptr;
    const int nbu = ceil_div(op.ntiles, kConsumerTiles);   // blocks of the two vector kernels
    // one column per mesh otherwise (an uneven batch, or one mesh too large for
    // every block to sum its partials): the fused step with a reduction block
    // per mesh, for a tuned shape or when chosen (shape 5)
    const bool fused_seg = !ssor && !fused && C == 1 && op.sp != nullptr && (o.spmm_shape == 0 || force_kind == 5);
    // its product keeps the slice columns in flight of the tuned sliced-ELLPACK shape
    const int seg_u = force_kind == 5 ? o.spmm_shape % 100
                      : (ch.kind == 2 || ch.kind == 3) && ch.a == 1 && ch.b == 8 ? 8 : 4;
    int64_t groups_done = 0;   // groups launched since the fused step's group count was cleared
    if (fused) {
        if (!w->snap_ring)
            PG_HIP(hipHostMalloc(reinterpret_cast<void**>(&w->snap_ring), sizeof(ColState) * kSnapRing));
        if (!w->gcount) PG_TRY(dalloc(&w->gcount, 1));
        hipLaunchKernelGGL(k_fill_rp, dim3(1), dim3(256), 0, s, 1, 0, w->gcount);
    }
    hipLaunchKernelGGL(k_init_state, dim3(ceil_div(nsc, 64)), dim3(64), 0, s, w->st, nsc,
                       o.inner_rtol, (int)sqmr);
    const bool prof = o.profile != 0;
    std::vector<hipEvent_t> evs;
    // a (start, end) pair the next SpMM dispatch timestamps, or nulls
    auto ev_pair = [&](SpmmArgs g) -> SpmmArgs {
        if (!prof) return g;
        (void)hipEventCreate(&g.e0);
        (void)hipEventCreate(&g.e1);
        evs.push_back(g.e0);
        evs.push_back(g.e1);
        return g;
    };
    auto residual = [&](int first) -> int {
        spmm_dispatch<double, 2>(ch64, op, w->st, SpmmArgs{w->X64, w->B64, w->R64, w->p0}, s);
        hipLaunchKernelGGL(k_reduce, dim3(nsc), dim3(1024), 0, s, op, w->p0, pp64, nullptr, 1, w->st,
                           (int)RED_RES, first);
        PG_HIP(hipGetLastError());
        return PETGEM_OK;
    };
    auto read_state = [&]() -> int {
        PG_HIP(hipMemcpyAsync(w->st_h, w->st, sizeof(ColState) * nsc, hipMemcpyDeviceToHost, s));
        PG_HIP(hipStreamSynchronize(s));
        return PETGEM_OK;
    };
    // |b| of every (segment, column)
    auto bnorms = [&]() -> int {
        hipLaunchKernelGGL(k_norm2, dim3(op.ntiles), dim3(256), 0, s, op, CP, w->B64, w->p0);
        hipLaunchKernelGGL(k_reduce, dim3(nsc), dim3(1024), 0, s, op, w->p0, 1, nullptr, 1, w->st,
                           (int)RED_RES, 1);
        PG_HIP(hipGetLastError());
        return PETGEM_OK;
    };
    PG_TRY(bnorms());
    hipLaunchKernelGGL(k_set_tol, dim3(ceil_div(nsc, 64)), dim3(64), 0, s, w->st, nsc, o.rtol);
    if (have_x0) {
        // scale every guess by the alpha minimising |b - alpha A x0|
        PG_TRY(residual(0));
        hipLaunchKernelGGL(k_x0_dots, dim3(op.ntiles), dim3(256), 0, s, op, CP, w->B64, w->R64, w->p0, w->p1);
        hipLaunchKernelGGL(k_reduce, dim3(nsc), dim3(1024), 0, s, op, w->p0, 1, w->p1, 1, w->st,
                           (int)RED_X0, 0);
        hipLaunchKernelGGL(k_scale_cols, dim3(op.ntiles), dim3(256), 0, s, op, CP, w->st, w->X64);
        PG_HIP(hipGetLastError());
    }
    // the true residual even for a zero start (taking |b| from k_norm2 instead,
    // a last-bit change of the first step's scale, made one column of a
    // 32-source block on the 6.9M-DOF marine mesh diverge in its second
    // refinement step)
    PG_TRY(residual(0));
    PG_TRY(read_state());
    std::vector<int> fallback(nsc, 0);
    if (have_x0) {
        bool redo = false;
        for (int k = 0; k < nsc; ++k) {
            const ColState& S = w->st_h[k];
            if (has_x0 && !(*has_x0)[k]) continue;
            if (!(S.rnorm64 < S.bnorm) && S.bnorm > 0.0) { fallback[k] = 1; redo = true; }
        }
        if (redo) {   // the rejected guesses restart from zero, the others stay
            PG_HIP(hipMemcpyAsync(w->flags, fallback.data(), sizeof(int) * nsc, hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL(k_zero_cols, dim3(op.ntiles), dim3(256), 0, s, op, CP, w->flags, w->X64);
            hipLaunchKernelGGL(k_init_state, dim3(ceil_div(nsc, 64)), dim3(64), 0, s, w->st, nsc,
                               o.inner_rtol, (int)sqmr);
            PG_TRY(bnorms());
            hipLaunchKernelGGL(k_set_tol, dim3(ceil_div(nsc, 64)), dim3(64), 0, s, w->st, nsc, o.rtol);
            PG_TRY(residual(0));
            PG_TRY(read_state());
        }
    }
    std::vector<double> x0res(nsc, 1.0);
    for (int k = 0; k < nsc; ++k)
        if (have_x0 && w->st_h[k].bnorm > 0 && (!has_x0 || (*has_x0)[k]))
            x0res[k] = fallback[k] ? 1.0 : w->st_h[k].rnorm64 / w->st_h[k].bnorm;

    // one inner iteration; a group of kCheck is captured as one graph
    // The inner-loop launches of an uneven batch cover only the tiles of the
    // meshes still iterating: after a check that finds the launched tiles at
    // least a quarter idle, the tile list is rebuilt from the active meshes
    // (and the graph captured anew). The reductions read only active meshes'
    // partials, all of which the list covers.
    Op opi = op;
    std::vector<int> tmap_h;
    int tgen = 0;   // generation of the launched tile list
    auto compact = [&]() -> int {
        if (!seg_tile_h || op.nseg <= 1 || C != 1) return PETGEM_OK;
        std::vector<int> list;
        for (int k = 0; k < op.nseg; ++k)
            if (w->st_h[k].active)
                for (int t = (*seg_tile_h)[k]; t < (*seg_tile_h)[k + 1]; ++t) list.push_back(t);
        if (list.empty() || 4 * (int64_t)list.size() > 3 * (int64_t)opi.nlaunch) return PETGEM_OK;
        if (!w->tmap) PG_TRY(dalloc(&w->tmap, (size_t)op.ntiles));
        tmap_h = std::move(list);
        PG_HIP(hipMemcpyAsync(w->tmap, tmap_h.data(), sizeof(int) * tmap_h.size(), hipMemcpyHostToDevice, s));
        PG_HIP(hipStreamSynchronize(s));   // tmap_h is reused by the next rebuild
        opi.tmap = w->tmap;
        opi.nlaunch = (int)tmap_h.size();
        ++tgen;
        return PETGEM_OK;
    };
    auto uncompact = [&]() {
        opi.tmap = nullptr;
        opi.nlaunch = op.ntiles;
    };
    // iteration k of a group: the fused step alternates its two state slots
    // with the parity of k (a group has an even count, so every group starts
    // and ends with the state in st)
    auto iteration = [&](int k) {
        if (fused) {
            const bool odd = (k & 1) != 0;
            ColState* sa = odd ? w->st2 : w->st;   // read by the product and the step
            ColState* sb = odd ? w->st : w->st2;   // written by the step
            const SpmmArgs g = ev_pair(SpmmArgs{w->P, nullptr, w->Q, w->p0});
            if (fused_u == 4)
                launch_timed_b(k_spmm_spb<4, kSpbWaves>, dim3(nspb), dim3(64 * kSpbWaves), s, g.e0, g.e1, opi,
                               (const ColState*)sa, (const float2*)w->P, w->Q, (const float2*)w->R, dinv, w->p0);
            else
                launch_timed_b(k_spmm_spb<8, kSpbWaves>, dim3(nspb), dim3(64 * kSpbWaves), s, g.e0, g.e1, opi,
                               (const ColState*)sa, (const float2*)w->P, w->Q, (const float2*)w->R, dinv, w->p0);
            // the step reads the previous step's partials from one half of p1,
            // p2 and writes its own to the other (its blocks run concurrently)
            const double2* gin = odd ? w->p1 + nst : w->p1;
            const double2* rin = odd ? w->p2 + nst : w->p2;
            double2* gout = odd ? w->p1 : w->p1 + nst;
            double2* rout = odd ? w->p2 : w->p2 + nst;
            hipLaunchKernelGGL(k_step1<kStepTiles>, dim3(nst), dim3(256), 0, s, op, (const ColState*)sa, sb,
                               (const double2*)w->p0, nspb, gin, rin, nst, w->R, (const float2*)w->Q, dinv,
                               w->P, w->Xi, gout, rout, k == kCheck - 1 ? w->snap_ring : nullptr, w->gcount);
            return;
        }
        if (fused_seg) {
            const SpmmArgs g = ev_pair(SpmmArgs{w->P, nullptr, w->Q, w->p0});
            if (seg_u == 8)
                launch_timed(k_spmm_spbs<8>, dim3(opi.nlaunch), s, g.e0, g.e1, opi, (const ColState*)w->st,
                             (const float2*)w->P, w->Q, (const float2*)w->R, w->p0);
            else
                launch_timed(k_spmm_spbs<4>, dim3(opi.nlaunch), s, g.e0, g.e1, opi, (const ColState*)w->st,
                             (const float2*)w->P, w->Q, (const float2*)w->R, w->p0);
            hipLaunchKernelGGL(k_red_seg, dim3(op.nseg), dim3(1024), 0, s, op, w->st, (const double2*)w->p0,
                               (const double2*)w->p1, (const double2*)w->p2);
            hipLaunchKernelGGL(k_step_seg, dim3(opi.nlaunch), dim3(256), 0, s, opi, (const ColState*)w->st, w->R,
                               (const float2*)w->Q, w->P, w->Xi, w->p1, w->p2);
            return;
        }
        if (eis) {
            // p = r + beta p; t = U1^-1 p (into Z)
            eis_upass(*sq, opi, w->st, w->R, w->P, w->Z, omega, s, prof ? &evs : nullptr);
            const int64_t cse = (int64_t)op.ntiles * ppE;
            eis_lpass(*sq, opi, w->st, w->P, w->Z, w->Q, omega, w->pe, cse, s);   // y (into Q), p^T (t + y)
            hipLaunchKernelGGL(k_reduce_cm, dim3(C), dim3(1024), 0, s, (const double2*)w->pe, neis, cse,
                               (const double2*)nullptr, 0, (int64_t)0, w->st, (int)RED_ALPHA);
            hipLaunchKernelGGL(k_eis_update, dim3(opi.nlaunch), dim3(256), 0, s, opi, CP, (const ColState*)w->st,
                               (const float2*)w->Z, (const float2*)w->Q, w->R, w->Xi, xq, omega, w->p1, w->p2);
            hipLaunchKernelGGL(k_reduce_cm, dim3(C), dim3(1024), 0, s, (const double2*)w->p1, op.ntiles,
                               (int64_t)op.ntiles, (const double2*)w->p2, op.ntiles, (int64_t)op.ntiles, w->st,
                               (int)RED_BETA);
            return;   // p = r + beta p in the next iteration's U pass
        }
        spmm_dispatch<float, 1>(ch, opi, w->st, ev_pair(SpmmArgs{w->P, nullptr, w->Q, w->p0}), s);
        if (in_consumer) {
            hipLaunchKernelGGL(k_update_p, dim3(nbu), dim3(256), 0, s, op, CP, kConsumerTiles, w->st, w->st2,
                               w->p0, op.ntiles * ppS, w->R, w->Z, w->Q, dinv, w->p1, w->p2);
            hipLaunchKernelGGL(k_pupdate_p, dim3(nbu), dim3(256), 0, s, op, CP, kConsumerTiles, w->st2, w->st,
                               w->p1, w->p2, nbu, w->Z, w->P, w->Xi);
        } else {
            hipLaunchKernelGGL(k_reduce, dim3(nsc), dim3(1024), 0, s, op, w->p0, ppS, nullptr, 1, w->st,
                               (int)RED_ALPHA, 0);
            hipLaunchKernelGGL(k_update, dim3(opi.nlaunch), dim3(256), 0, s, opi, CP, w->st, w->R, w->Z, w->Q,
                               dinv, w->p1, w->p2, ssor ? 0 : 1);
            if (ssor) {
                ssor_sweeps(*sq, opi, w->st, w->R, w->Z, omega, s);
                hipLaunchKernelGGL(k_rz, dim3(opi.nlaunch), dim3(256), 0, s, opi, CP, (const ColState*)w->st,
                                   (const float2*)w->R, (const float2*)w->Z, (float2*)nullptr, w->p1);
            }
            hipLaunchKernelGGL(k_reduce, dim3(nsc), dim3(1024), 0, s, op, w->p1, 1, w->p2, 1, w->st,
                               (int)RED_BETA, 0);
            hipLaunchKernelGGL(k_pupdate, dim3(opi.nlaunch), dim3(256), 0, s, opi, CP, w->st, w->Z, w->P, w->Xi,
                               xq);
        }
    };
    auto group = [&]() {
        for (int k = 0; k < kCheck; ++k) iteration(k);
    };
    const bool use_graph = o.use_graph && !prof;
    // (re)capture the graph of ng groups; every graph is dropped whenever an
    // argument baked into them changed
    auto ensure_graph = [&](int ng) -> int {
        if (!use_graph) return PETGEM_OK;
        std::vector<char> sig;
        auto put = [&](const void* p, size_t nb) {
            const char* c = static_cast<const char*>(p);
            sig.insert(sig.end(), c, c + nb);
        };
        put(&opi, sizeof(opi));
        const void* ptrs[17] = {w->Xi, w->R, w->Z, w->P, w->Q, w->p0, w->p1, w->p2, w->st, w->st2, dinv,
                                w->snap_ring, w->gcount, sq ? (const void*)sq->row : nullptr,
                                sq ? (const void*)sq->lK : nullptr, eis ? (const void*)w->pe : nullptr,
                                (const void*)xq};
        put(ptrs, sizeof(ptrs));
        int chv[12] = {ch.kind, ch.a, ch.b, (int)in_consumer, opi.tmap ? tgen : 0, (int)fused, fused_u, (int)fused_seg,
                       seg_u, (int)ssor, ssor ? (int)(o.omega * 1e6) : 0, ppE};
        put(chv, sizeof(chv));
        if (w->graph_sig != sig) w->release_graph();
        if (w->graphs[ng - 1] != nullptr) return PETGEM_OK;
        if (!w->graph_stream) PG_HIP(hipStreamCreateWithFlags(&w->graph_stream, hipStreamNonBlocking));
        hipGraph_t g;
        hipStream_t caller = s;
        s = w->graph_stream;
        PG_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        for (int k = 0; k < ng; ++k) group();
        hipError_t ce = hipStreamEndCapture(s, &g);
        s = caller;
        if (ce != hipSuccess) {
            set_error(std::string("graph capture: ") + hipGetErrorString(ce));
            return PETGEM_HIP_ERROR;
        }
        hipError_t ie = hipGraphInstantiate(&w->graphs[ng - 1], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) {
            set_error(std::string("graph instantiate: ") + hipGetErrorString(ie));
            return PETGEM_HIP_ERROR;
        }
        w->graph_sig = sig;
        return PETGEM_OK;
    };

    int total_inner = 0, steps = 0, strikes = 0;
    const char* why = "";
    int status = PETGEM_OK;
    const int max_steps = 60;
    double prev_worst = 1e300;
    while (true) {
        int n_outer = 0;
        bool nonfinite = false;
        for (int k = 0; k < nsc; ++k) {
            n_outer += w->st_h[k].outer;
            if (!std::isfinite(w->st_h[k].rnorm64)) nonfinite = true;
        }
        if (nonfinite) { status = PETGEM_NONFINITE; break; }
        if (n_outer == 0) break;
        // stagnation: the worst relative residual must at least halve per step
        double worst = 0.0;
        for (int k = 0; k < nsc; ++k)
            if (w->st_h[k].outer && w->st_h[k].bnorm > 0)
                worst = std::max(worst, w->st_h[k].rnorm64 / w->st_h[k].bnorm);
        strikes = worst > 0.5 * prev_worst ? strikes + 1 : 0;
        prev_worst = worst;
        if (strikes >= 3) {
            status = PETGEM_NOT_CONVERGED;
            why = "stagnated (the worst residual did not halve in 3 refinement steps)";
            break;
        }
        if (steps >= max_steps || total_inner >= o.max_iter) {
            status = PETGEM_NOT_CONVERGED;
            why = steps >= max_steps ? "reached its refinement step limit" : "reached max_iter";
            break;
        }
        // inner complex64 COCG on A d = r64 / |r64|
        hipLaunchKernelGGL(k_inner_init, dim3(op.ntiles), dim3(256), 0, s, op, CP, w->R64, w->st, dinv, w->Xi,
                           w->R, w->Z, w->P, w->p1, w->p2);
        if (eis) {    // y0 = L1^-1 r0, then the split residual r = D~ y0, p = r; rho and its norm
            ssor_pass(*sq, op, nullptr, w->R, w->Q, omega, false, false, s);
            hipLaunchKernelGGL(k_eis_init, dim3(op.ntiles), dim3(256), 0, s, op, CP, (const ColState*)w->st,
                               (const float2*)w->Q, w->R, w->P, omega, w->p1, w->p2);
        } else if (ssor) {   // z = M^-1 r, p = z and the r^T z partials by the sweeps
            ssor_sweeps(*sq, op, nullptr, w->R, w->Z, omega, s);
            hipLaunchKernelGGL(k_rz, dim3(op.ntiles), dim3(256), 0, s, op, CP, (const ColState*)w->st,
                               (const float2*)w->R, (const float2*)w->Z, w->P, w->p1);
        }
        hipLaunchKernelGGL(k_reduce, dim3(nsc), dim3(1024), 0, s, op, w->p1, 1, w->p2, 1, w->st,
                           (int)(eis ? RED_INIT_REL : RED_INIT), 0);
        // Groups of kCheck iterations run between host checks; the number of
        // groups in a row follows the observed decrease of the worst active
        // residual (half the predicted need, at most kMaxGroups), so that the
        // readbacks are few while little runs past convergence.
        int inner = 0, groups = 1, next_print = 512;
        double prev_gap = -1.0;
        uncompact();
        // A single system keeps one more batch of iteration groups queued while
        // the host reads the state after the previous batch, so the GPU does
        // not idle during the check; a batch queued after convergence finds
        // every column inactive and changes nothing. An uneven batch checks
        // synchronously: a check may rebuild its tile list.
        const bool overlap = use_graph && !(seg_tile_h && op.nseg > 1);
        ColState* snap[2] = {w->st_h, w->st_h2};
        int cur = 0;
        // the fused step writes the state of every group's end into the host
        // ring itself; a batch's state is then in the slot of its last group
        // (the at most kMaxGroups groups queued behind it cannot reach that
        // slot again)
        static_assert(kSnapRing > 2 * kMaxGroups, "a queued batch must not overwrite the slot being read");
        // A single system launches a batch of n groups as one graph of n
        // groups: the kernels inside one graph follow each other without the
        // gap that separates two graph launches. An uneven batch recaptures
        // its graph after each rebuild of its tile list, so it keeps to the
        // one-group graph, whose capture is cheapest.
        const int ng_max = overlap ? kMaxGroups : 1;
        auto launch_batch = [&](int n, int slot) -> int {
            if (use_graph) {
                for (int left = n; left > 0;) {
                    const int ng = std::min(left, ng_max);
                    PG_TRY(ensure_graph(ng));
                    PG_HIP(hipGraphLaunch(w->graphs[ng - 1], s));
                    left -= ng;
                }
            } else {
                for (int g = 0; g < n; ++g) group();
            }
            inner += kCheck * n;
            if (fused) {
                groups_done += n;
                snap[slot] = w->snap_ring + ((groups_done - 1) & (kSnapRing - 1));
            } else {
                snap[slot] = slot ? w->st_h2 : w->st_h;
                PG_HIP(hipMemcpyAsync(snap[slot], w->st, sizeof(ColState) * nsc, hipMemcpyDeviceToHost, s));
            }
            PG_HIP(hipEventRecord(w->snap_ev[slot], s));
            return PETGEM_OK;
        };
        PG_TRY(launch_batch(groups, cur));
        int queued = groups;   // groups of the batch that snap[cur] follows
        double need = -1.0;    // half the predicted groups to convergence (-1: unknown)
        while (true) {
            int ahead = 0;
            if (overlap) {
                if (need < 0.0) ahead = 1;
                else if (need > queued) ahead = (int)std::min<double>(kMaxGroups, std::max(1.0, need - queued));
                ahead = std::min(ahead, std::max(0, (o.max_iter - total_inner - inner) / kCheck));
                if (ahead > 0) PG_TRY(launch_batch(ahead, cur ^ 1));
            }
            PG_HIP(hipEventSynchronize(w->snap_ev[cur]));
            const ColState* sv = snap[cur];
            int act = 0;
            double gap = 0.0;   // worst log(|r|^2 / tol^2) over the active columns
            for (int k = 0; k < nsc; ++k) {
                const ColState& S = sv[k];
                if (!S.active) continue;
                ++act;
                if (S.rn2 > 0.0 && S.inner_tol2 > 0.0)
                    gap = std::max(gap, std::log(S.rn2 / (S.inner_tol2 * S.rn2_0)));
            }
            if (o.verbose && inner >= next_print) {
                double worst = 0.0;
                int kw = -1;
                for (int k = 0; k < nsc; ++k)
                    if (sv[k].active && sv[k].rn2 >= worst) { worst = sv[k].rn2; kw = k; }
                fprintf(stderr, "[petgem]   inner %d: %d active, worst inner residual %.3e (column %d, its best "
                        "%.3e at %d), %.0f ms\n", inner, act, std::sqrt(worst), kw,
                        kw >= 0 ? std::sqrt(sv[kw].rn2_best) : 0.0, kw >= 0 ? sv[kw].k_best : 0, t_all.ms());
                fflush(stderr);
                next_print += 512;
            }
            if (act == 0 || total_inner + inner >= o.max_iter) break;
            need = -1.0;
            if (prev_gap > 0.0 && gap < prev_gap && std::isfinite(gap)) need = 0.5 * gap * queued / (prev_gap - gap);
            prev_gap = gap;
            if (ahead > 0) {   // the next state is already on its way
                cur ^= 1;
                queued = ahead;
                continue;
            }
            PG_TRY(compact());
            groups = need < 0.0 ? 1 : (int)std::min<double>(kMaxGroups, std::max(1.0, need));
            groups = std::max(1, std::min(groups, (o.max_iter - total_inner - inner) / kCheck));
            PG_TRY(launch_batch(groups, cur));
            queued = groups;
        }
        total_inner += inner;
        hipLaunchKernelGGL(k_ir_update, dim3(op.ntiles), dim3(256), 0, s, op, CP, w->st, w->Xi,
                           (const float2*)xq, eis ? 1 : 0, w->X64);
        PG_TRY(residual(0));
        PG_TRY(read_state());
        ++steps;
        if (o.verbose) {
            double worst = 0.0;
            int left = 0, stalls = 0;
            for (int k = 0; k < nsc; ++k) {
                if (w->st_h[k].bnorm > 0) worst = std::max(worst, w->st_h[k].rnorm64 / w->st_h[k].bnorm);
                left += w->st_h[k].outer;
                stalls += w->st_h[k].stalled;
            }
            fprintf(stderr, "[petgem] COCG refinement step %d: %d inner iterations, worst true residual "
                            "%.3e, %d of %d columns left, %d inner solves stopped by the stagnation guard, "
                            "%.0f ms\n", steps, inner, worst, left, nsc, stalls, t_all.ms());
            if (o.verbose >= 2)   // each column's inner solve of this step
                for (int k = 0; k < nsc; ++k) {
                    const ColState& S = w->st_h[k];
                    const double r0 = S.rn2_0 > 0.0 ? S.rn2_0 : 1.0;
                    fprintf(stderr, "[petgem]     column %d: %d inner iterations, best %.2e at %d, last %.2e, "
                                    "true residual %.3e, stops by the guards so far %d\n", k, S.kin,
                            std::sqrt(S.rn2_best / r0), S.k_best, std::sqrt(S.rn2 / r0),
                            S.bnorm > 0 ? S.rnorm64 / S.bnorm : 0.0, S.stalled);
                }
            fflush(stderr);
        }
    }
    double t_solve = t_all.ms();
    double spmv_ms = 0.0;
    int spmv_n = 0;
    if (prof && !evs.empty()) {
        (void)hipEventSynchronize(evs.back());
        for (size_t i = 0; i + 1 < evs.size(); i += 2) {
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, evs[i], evs[i + 1]);
            spmv_ms += ms;
            ++spmv_n;
        }
        for (auto e : evs) (void)hipEventDestroy(e);
    }
    for (int k = 0; k < nsc; ++k) {
        petgem_stats* st = stv[k];
        if (!st) continue;
        const ColState& S = w->st_h[k];
        st->iters = S.iters;
        st->ir_steps = steps;
        st->used_fallback = fallback[k];
        st->rel_residual = S.bnorm > 0 ? S.rnorm64 / S.bnorm : 0.0;
        st->b_norm = S.bnorm;
        st->x0_rel_residual = x0res[k];
        st->t_solve_ms = t_solve;
        st->spmv_ms = spmv_ms;
        st->spmv_launches = spmv_n;
        st->spmv_shape = fused ? 40100 + fused_u : fused_seg ? 50100 + seg_u
                         : eis ? 70000 + 100 * eis_lpr(C) + (C <= 64 ? 1 : C <= 128 ? 2 : 4)
                               : 10000 * ch.kind + 100 * ch.a + ch.b;
        st->status = S.outer ? (std::isfinite(S.rnorm64) ? PETGEM_NOT_CONVERGED : PETGEM_NONFINITE) : PETGEM_OK;
        if (st->status != PETGEM_OK && status == PETGEM_OK) status = st->status;
    }
    if (status == PETGEM_NOT_CONVERGED) {
        int kw = 0;
        double worst = -1.0;
        for (int k = 0; k < nsc; ++k)
            if (w->st_h[k].outer && w->st_h[k].bnorm > 0 && w->st_h[k].rnorm64 / w->st_h[k].bnorm > worst) {
                worst = w->st_h[k].rnorm64 / w->st_h[k].bnorm;
                kw = k;
            }
        char msg[256];
        snprintf(msg, sizeof msg, "COCG refinement %s before rtol %.1e: %d steps, %d inner iterations, "
                 "worst relative residual %.3e (segment %d, column %d)", why, o.rtol, steps, total_inner,
                 worst, kw / C, kw % C);
        set_error(msg);
    }
    if (status == PETGEM_NONFINITE) set_error("non-finite value in the COCG recurrence");
    return status;
}

// ------------------------------------------- block COCG
// O'Leary's block conjugate gradient carried over to the complex-symmetric
// bilinear form u^T v (not in the paper; the columns are sources of one
// frequency, so they share A): the C columns share one block Krylov space.
// With P the block of search directions (orthonormal columns in the
// Hermitian product, dependent directions dropped), Q = A P and G = P^T Q:
//   alpha = G^-1 (P^T R)      X += P alpha     R -= Q alpha     (P^T R = 0)
//   Z = D^-1 R                beta = -G^-1 (Q^T Z)              (P^T A P_new = 0)
//   P~ = Z + P beta           Gamma = P~^H P~ = R_c^H R_c (Cholesky with
//   diagonal pivoting; a pivot below kDefl^2 of the largest diagonal ends it:
//   rank r)                   P = P~ Pi R_c^-1 (first r columns, the rest zero).
// Everything runs in double precision: in complex64 the block recurrence
// loses conjugacy within some tens of iterations on the 3,032-unknown model
// (the residual grows by orders of magnitude at any drop threshold tried,
// 1e-3 to 1e-7), while in complex128 it converges. The recursive residual
// stops the iteration; the solve then restarts from the true residual until
// it meets rtol. A direction is dropped when it is nearly dependent on the
// others: the Gram matrix is scaled to a unit diagonal before the pivoted
// Cholesky, whose pivot must stay above kDefl^2 (columns that are small but
// independent are kept: dropping them breaks the conjugacy of later blocks;
// keeping directions dependent to 1e-10 made the change of basis blow up on
// 32 closely spaced sources).
constexpr int kBlkTiles = 8;        // tiles per block of the Gram kernels
constexpr double kDefl = 1e-7;      // relative norm of a nearly dependent direction

// out[b][m][i][j] = sum over the rows of block b of U_m[r][i] V_m[r][j]
// (conj(U_m) for CONJ), m < nprod, in double.
template <bool CONJ>
__global__ void __launch_bounds__(256)
k_bgram(Op op, const double2* __restrict__ U1, const double2* __restrict__ V1, const double2* __restrict__ U2,
        const double2* __restrict__ V2, int nprod, double2* __restrict__ out) {
    const int C = op.C, CC = C * C;
    const int r0 = blockIdx.x * kBlkTiles * kTR;
    const int r1 = min(r0 + kBlkTiles * kTR, op.nrow_valid);
    for (int e = threadIdx.x; e < nprod * CC; e += 256) {
        const int m = e / CC, ij = e % CC, i = ij / C, j = ij % C;
        const double2* U = m ? U2 : U1;
        const double2* V = m ? V2 : V1;
        double2 a = make_double2(0.0, 0.0);
        for (int r = r0; r < r1; ++r) {
            const double2 u = U[(size_t)r * C + i], v = V[(size_t)r * C + j];
            const double ux = u.x, uy = CONJ ? -(double)u.y : (double)u.y;
            a.x += ux * v.x - uy * v.y;
            a.y += ux * v.y + uy * v.x;
        }
        out[(size_t)blockIdx.x * nprod * CC + e] = a;
    }
}

// res[e] = sum over the nb blocks of part[b][e] (fixed order: strided per
// thread, then the waves), one workgroup per entry e < ne.
__global__ void __launch_bounds__(256)
k_bred(int nb, int ne, const double2* __restrict__ part, double2* __restrict__ res) {
    __shared__ double2 ws[4];
    const int e = blockIdx.x;
    double2 a = make_double2(0.0, 0.0);
    for (int b = threadIdx.x; b < nb; b += 256) a = cadd(a, part[(size_t)b * ne + e]);
    a.x = wave_sum(a.x);
    a.y = wave_sum(a.y);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) res[e] = cadd(cadd(ws[0], ws[1]), cadd(ws[2], ws[3]));
}

// State of the block iteration on the device.
struct BlkState {
    int rank;        // directions in P (its first `rank` columns)
    int stop;        // breakdown: G singular on the kept directions
    int iters;
};

// Columns that have met rtol take no further part: their residual is zeroed
// (their alpha then stays zero and X keeps its converged value).
__global__ void __launch_bounds__(256)
k_bzero_done(Op op, int CP, const ColState* __restrict__ st, double2* __restrict__ R) {
    const int tile = blockIdx.x, C = op.C;
    const int c = threadIdx.x % CP, slot = threadIdx.x / CP, RPB = 256 / CP;
    if (c >= C || st[c].outer) return;
    for (int r0 = 0; r0 < kTR; r0 += RPB) {
        const int i = tile * kTR + r0 + slot;
        if (i >= op.ntiles * kTR) break;
        R[(size_t)i * C + c] = make_double2(0.0, 0.0);
    }
}

// Small dense algebra of the block iteration, one workgroup of 64 threads,
// complex double in LDS (C <= 32).
//  mode 0: alpha = G^-1 H (G = gram[0], H = gram[1]), rows >= rank zero.
//  mode 1: beta = -G^-1 W (G kept from mode 0 in g_keep, W = gram[0]).
//  mode 2: T from Gamma = gram[0] (Hermitian): pivoted Cholesky, new rank.
constexpr int kBlkMax = 32;
__global__ void __launch_bounds__(64)
k_bsmall(int C, int mode, const double2* __restrict__ gram, double2* __restrict__ g_keep,
         double2* __restrict__ outm, BlkState* __restrict__ bs) {
    __shared__ double2 a[kBlkMax][2 * kBlkMax];
    __shared__ int piv[kBlkMax];
    __shared__ int s_rank, s_stop;
    const int t = threadIdx.x;
    if (t == 0) { s_rank = bs->rank; s_stop = bs->stop; }
    __syncthreads();
    const int r = s_rank;
    if (s_stop) return;
    if (mode == 0 || mode == 1) {
        // [G_rr | RHS_r,:] with RHS = H (mode 0) or -W (mode 1)
        const double2* G = mode == 0 ? gram : g_keep;
        const double2* Rhs = mode == 0 ? gram + C * C : gram;
        for (int e = t; e < r * (r + C); e += 64) {
            const int i = e / (r + C), j = e % (r + C);
            double2 v = j < r ? G[i * C + j] : Rhs[i * C + (j - r)];
            if (j >= r && mode == 1) v = make_double2(-v.x, -v.y);
            a[i][j] = v;
        }
        if (mode == 0)
            for (int e = t; e < C * C; e += 64) g_keep[e] = gram[e];
        __syncthreads();
        double gmax = 0.0;
        for (int i = 0; i < r; ++i)
            for (int j = 0; j < r; ++j) gmax = fmax(gmax, cabs2(a[i][j]));
        for (int k = 0; k < r; ++k) {
            if (t == 0) {
                int p = k;
                for (int i = k + 1; i < r; ++i)
                    if (cabs2(a[i][k]) > cabs2(a[p][k])) p = i;
                piv[k] = p;
                if (!(cabs2(a[p][k]) > 1e-20 * gmax)) s_stop = 1;
            }
            __syncthreads();
            if (s_stop) break;
            const int p = piv[k];
            if (p != k)
                for (int j = t; j < r + C; j += 64) {
                    const double2 x = a[k][j];
                    a[k][j] = a[p][j];
                    a[p][j] = x;
                }
            __syncthreads();
            const double2 inv = cdiv(make_double2(1.0, 0.0), a[k][k]);
            for (int e = t; e < (r - k - 1) * (r + C); e += 64) {
                const int i = k + 1 + e / (r + C), j = e % (r + C);
                if (j <= k) continue;
                const double2 f = cmul(a[i][k], inv);
                a[i][j] = csub(a[i][j], cmul(f, a[k][j]));
            }
            __syncthreads();
        }
        if (s_stop) {
            if (t == 0) bs->stop = 1;
            return;
        }
        // back substitution, one right-hand column per thread
        for (int j = t; j < C; j += 64) {
            for (int i = r - 1; i >= 0; --i) {
                double2 v = a[i][r + j];
                for (int k = i + 1; k < r; ++k) v = csub(v, cmul(a[i][k], a[k][r + j]));
                a[i][r + j] = cdiv(v, a[i][i]);
            }
        }
        __syncthreads();
        for (int e = t; e < C * C; e += 64) {
            const int i = e / C, j = e % C;
            outm[e] = i < r ? a[i][r + j] : make_double2(0.0, 0.0);
        }
        return;
    }
    // mode 2: pivoted Cholesky of Gamma (C x C Hermitian) scaled to a unit
    // diagonal, S Gamma S = L L^H (S = diag(Gamma)^-1/2; zero columns stay out)
    __shared__ double sc[kBlkMax];
    if (t < C) sc[t] = gram[t * C + t].x > 0.0 ? 1.0 / sqrt(gram[t * C + t].x) : 0.0;
    __syncthreads();
    for (int e = t; e < C * C; e += 64) a[e / C][e % C] = cscale(gram[e], sc[e / C] * sc[e % C]);
    if (t < C) piv[t] = t;
    __syncthreads();
    if (t == 0) {
        const double dmax = 1.0;
        int rank = 0;
        for (int k = 0; k < C; ++k) {
            int p = k;
            for (int i = k + 1; i < C; ++i)
                if (a[i][i].x > a[p][p].x) p = i;
            if (!(a[p][p].x > kDefl * kDefl * dmax)) break;
            if (p != k) {   // symmetric swap of rows and columns k, p
                for (int j = 0; j < C; ++j) { const double2 x = a[k][j]; a[k][j] = a[p][j]; a[p][j] = x; }
                for (int i = 0; i < C; ++i) { const double2 x = a[i][k]; a[i][k] = a[i][p]; a[i][p] = x; }
                const int q = piv[k]; piv[k] = piv[p]; piv[p] = q;
            }
            const double l = sqrt(a[k][k].x);
            a[k][k] = make_double2(l, 0.0);
            for (int i = k + 1; i < C; ++i) a[i][k] = cscale(a[i][k], 1.0 / l);
            for (int i = k + 1; i < C; ++i)
                for (int j = k + 1; j <= i; ++j) {
                    a[i][j] = csub(a[i][j], cmul(a[i][k], cconj(a[j][k])));
                    a[j][i] = cconj(a[i][j]);
                }
            rank = k + 1;
        }
        s_rank = rank;
    }
    __syncthreads();
    const int rk = s_rank;
    // T = Pi[:, :rk] (L_rk^H)^-1: column j of the inverse of the upper
    // triangular R = L^H, one column per thread
    __shared__ double2 rinv[kBlkMax][kBlkMax];
    for (int j = t; j < rk; j += 64) {
        for (int i = rk - 1; i >= 0; --i) {
            double2 v = make_double2(i == j ? 1.0 : 0.0, 0.0);
            for (int k = i + 1; k < rk; ++k) v = csub(v, cmul(cconj(a[k][i]), rinv[k][j]));
            rinv[i][j] = cdiv(v, cconj(a[i][i]));
        }
    }
    __syncthreads();
    for (int e = t; e < C * C; e += 64) {
        const int i = e / C, j = e % C;   // T[i][j]: row i of P~ into column j of P
        double2 v = make_double2(0.0, 0.0);
        if (j < rk)
            for (int k = 0; k < rk; ++k)
                if (piv[k] == i) v = cscale(rinv[k][j], sc[i]);
        outm[e] = v;
    }
    if (t == 0) bs->rank = rk;
}

// Row updates of the block iteration: Y_c = A_c + sgn sum_k B_k M[k][c]
// (A, B, Y null-able as stated; M in LDS). With zout: also z = D^-1 Y (the
// column's Jacobi) into zout and the partials |Y_c|^2 per tile (part).
__global__ void __launch_bounds__(256)
k_bmul(Op op, int CP, const double2* __restrict__ Ain, const double2* __restrict__ Bv,
       const double2* __restrict__ Mm, double sgn, double2* __restrict__ Y, double2* __restrict__ zout,
       double2* __restrict__ part, const BlkState* __restrict__ bs) {
    __shared__ double2 Ms[kBlkMax * kBlkMax];
    __shared__ double2 ra[256], rb[256];
    const int C = op.C;
    // after a breakdown the small matrices are stale: leave everything as it is
    // until the host restarts the block from the true residual
    if (bs && bs->stop) return;
    for (int e = threadIdx.x; e < C * C; e += 256) Ms[e] = Bv ? Mm[e] : make_double2(0.0, 0.0);
    __syncthreads();
    const int tile = blockIdx.x;
    const int c = threadIdx.x % CP, slot = threadIdx.x / CP, RPB = 256 / CP;
    double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
    if (c < C) {
        const double wmu = op.wmu[c];
        for (int r0 = 0; r0 < kTR; r0 += RPB) {
            const int i = tile * kTR + r0 + slot;
            if (i >= op.nrow_valid) break;
            double2 acc = make_double2(0.0, 0.0);
            if (Bv) {
                const double2* br = Bv + (size_t)i * C;
                for (int k = 0; k < C; ++k) acc = cadd(acc, cmul(br[k], Ms[k * C + c]));   // rows past the rank are zero
            }
            const size_t o = (size_t)i * C + c;
            const double2 av = Ain ? Ain[o] : make_double2(0.0, 0.0);
            const double2 y = make_double2(av.x + sgn * acc.x, av.y + sgn * acc.y);
            Y[o] = y;
            if (zout) {
                // z = y / (Kd - i wmu Md)
                const double dr = op.Kd[i], di = -wmu * op.Md[i];
                const double inv = 1.0 / (dr * dr + di * di);
                zout[o] = make_double2((y.x * dr + y.y * di) * inv, (y.y * dr - y.x * di) * inv);
                b.x += y.x * y.x + y.y * y.y;
            }
        }
    }
    if (!part) return;
    cp_sum2(a, b, CP, ra, rb);
    if ((int)threadIdx.x < C && (int)threadIdx.x < CP) part[(size_t)tile * C + threadIdx.x] = rb[threadIdx.x];
}

}  // namespace

int spmm_candidate_codes(int C, bool sliced, int32_t* out, int cap) {
    const auto v = candidates(C, sliced);
    int n = 0;
    for (const SpmmChoice& c : v) {
        if (out && n < cap) out[n] = 10000 * c.kind + 100 * c.a + c.b;
        ++n;
    }
    return n;
}

namespace {

// Block COCG in double precision (one mesh, C <= 32 columns of one
// frequency, zero initial guesses): block iterations on the true residual
// until every recursive residual is 0.3 rtol |b| or less, then a restart
// from the true residual while any column misses rtol. The bilinear form
// P^T A P is indefinite, so the block recurrence can lose conjugacy: with
// more than a few nearly dependent sources (closely spaced dipoles) the
// recursive residuals grow without bound, while the same code converges on a
// real symmetric positive definite operator. Once the worst recursive
// residual (relative to its target) is ten times the lowest it reached in
// this restart, or after kBlkRestarts restarts, the block phase ends with
// *handoff set and X64 holding its iterate, from which the caller finishes
// the columns as independent COCG.
constexpr double kBlkGrowth = 100.0;   // squared growth of the worst recursive residual
constexpr int kBlkRestarts = 20;
int bcocg_solve(BlockWork* w, const Op& op, int64_t nnz, const petgem_opts& o, hipStream_t s,
                std::vector<petgem_stats*>& stv, bool* handoff, int* block_iters) {
    const int C = op.C, CP = cp_of(C), CC = C * C;
    Timer t_all;
    SpmmTuned tu;
    PG_TRY(tune_spmm(w, op, nnz, s, tu, o.verbose != 0));
    const SpmmChoice ch64 = tu.csr;   // a CSR shape (the complex128 product)
    const int pp64 = spmm_slots(ch64);
    const int nblk = ceil_div(op.ntiles, kBlkTiles);
    const size_t nv = (size_t)op.ntiles * kTR * C;
    double2 *gpart = nullptr, *gram = nullptr, *gkeep = nullptr, *mat = nullptr, *norms = nullptr;
    double2 *P = nullptr, *Q = nullptr, *Z = nullptr;
    BlkState* bs = nullptr;
    struct Frees {
        double2** p[8];
        BlkState** b;
        ~Frees() { for (auto q : p) dfree(*q); dfree(*b); }
    } frees{{&gpart, &gram, &gkeep, &mat, &norms, &P, &Q, &Z}, &bs};
    PG_TRY(dalloc(&gpart, (size_t)nblk * 2 * CC));
    PG_TRY(dalloc(&gram, (size_t)2 * CC));
    PG_TRY(dalloc(&gkeep, (size_t)CC));
    PG_TRY(dalloc(&mat, (size_t)CC));
    PG_TRY(dalloc(&norms, (size_t)C));
    PG_TRY(dalloc(&P, nv));
    PG_TRY(dalloc(&Q, nv));
    PG_TRY(dalloc(&Z, nv));
    PG_TRY(dalloc(&bs, 1));
    hipLaunchKernelGGL(k_init_state, dim3(ceil_div(C, 64)), dim3(64), 0, s, w->st, C, o.inner_rtol, 0);
    hipLaunchKernelGGL(k_set_live, dim3(ceil_div(C, 64)), dim3(64), 0, s, w->st2, C);   // every product column live
    auto residual = [&]() -> int {
        spmm_dispatch<double, 2>(ch64, op, w->st, SpmmArgs{w->X64, w->B64, w->R64, w->p0}, s);
        hipLaunchKernelGGL(k_reduce, dim3(C), dim3(1024), 0, s, op, w->p0, pp64, nullptr, 1, w->st, (int)RED_RES, 0);
        PG_HIP(hipGetLastError());
        return PETGEM_OK;
    };
    auto read_state = [&]() -> int {
        PG_HIP(hipMemcpyAsync(w->st_h, w->st, sizeof(ColState) * C, hipMemcpyDeviceToHost, s));
        PG_HIP(hipStreamSynchronize(s));
        return PETGEM_OK;
    };
    hipLaunchKernelGGL(k_norm2, dim3(op.ntiles), dim3(256), 0, s, op, CP, w->B64, w->p0);
    hipLaunchKernelGGL(k_reduce, dim3(C), dim3(1024), 0, s, op, w->p0, 1, nullptr, 1, w->st, (int)RED_RES, 1);
    hipLaunchKernelGGL(k_set_tol, dim3(ceil_div(C, 64)), dim3(64), 0, s, w->st, C, o.rtol);
    PG_TRY(residual());
    PG_TRY(read_state());
    auto gram_of = [&](bool conj, const double2* U1, const double2* V1, const double2* U2, const double2* V2,
                       int nprod) {
        if (conj)
            hipLaunchKernelGGL(k_bgram<true>, dim3(nblk), dim3(256), 0, s, op, U1, V1, U2, V2, nprod, gpart);
        else
            hipLaunchKernelGGL(k_bgram<false>, dim3(nblk), dim3(256), 0, s, op, U1, V1, U2, V2, nprod, gpart);
        hipLaunchKernelGGL(k_bred, dim3(nprod * CC), dim3(256), 0, s, nblk, nprod * CC, (const double2*)gpart,
                           gram);
    };
    auto bmul = [&](const double2* Ain, const double2* Bv, double sgn, double2* Y, double2* zout, double2* part) {
        hipLaunchKernelGGL(k_bmul, dim3(op.ntiles), dim3(256), 0, s, op, CP, Ain, Bv, (const double2*)mat, sgn, Y,
                           zout, part, (const BlkState*)bs);
    };
    auto small = [&](int mode) {
        hipLaunchKernelGGL(k_bsmall, dim3(1), dim3(64), 0, s, C, mode, (const double2*)gram, gkeep, mat, bs);
    };
    int restarts = 0, total = 0, status = PETGEM_OK;
    const char* why = "";
    std::vector<double2> nh(C);
    while (true) {
        int n_outer = 0;
        for (int k = 0; k < C; ++k) {
            const ColState& S = w->st_h[k];
            n_outer += S.outer;
            if (!std::isfinite(S.rnorm64)) { status = PETGEM_NONFINITE; break; }
        }
        if (status != PETGEM_OK || n_outer == 0) break;
        if (total >= o.max_iter) {
            status = PETGEM_NOT_CONVERGED;
            why = "reached max_iter";
            break;
        }
        if (restarts >= kBlkRestarts) { *handoff = true; break; }
        // the recursive residual of each column is to reach 0.3 rtol |b|
        std::vector<double> tol2(C);
        for (int k = 0; k < C; ++k) {
            const ColState& S = w->st_h[k];
            tol2[k] = S.outer ? (0.3 * S.tol_abs) * (0.3 * S.tol_abs) : 1e300;
        }
        // R = the true residual (R64) of the columns still above rtol; Z = D^-1 R;
        // P = Z T with P^H P = I
        hipLaunchKernelGGL(k_bzero_done, dim3(op.ntiles), dim3(256), 0, s, op, CP, (const ColState*)w->st, w->R64);
        BlkState b0{C, 0, 0};
        PG_HIP(hipMemcpyAsync(bs, &b0, sizeof(b0), hipMemcpyHostToDevice, s));
        bmul(w->R64, nullptr, 0.0, w->R64, Z, nullptr);
        gram_of(true, Z, Z, nullptr, nullptr, 1);
        small(2);
        bmul(nullptr, Z, 1.0, P, nullptr, nullptr);
        int it = 0;
        bool grew = false;
        double lowest = INFINITY;
        while (true) {
            for (int g = 0; g < kCheck; ++g) {
                spmm_dispatch<double, 1>(ch64, op, w->st2, SpmmArgs{P, nullptr, Q, w->p0}, s);   // Q = A P
                gram_of(false, P, Q, P, w->R64, 2);                 // G = P^T Q, H = P^T R
                small(0);                                           // alpha = G^-1 H
                bmul(w->X64, P, 1.0, w->X64, nullptr, nullptr);     // X += P alpha
                bmul(w->R64, Q, -1.0, w->R64, Z, w->p1);            // R -= Q alpha; Z = D^-1 R; |R|^2
                gram_of(false, Q, Z, nullptr, nullptr, 1);          // W = Q^T Z
                small(1);                                           // beta = -G^-1 W
                bmul(Z, P, 1.0, Q, nullptr, nullptr);               // P~ = Z + P beta (in Q)
                gram_of(true, Q, Q, nullptr, nullptr, 1);           // P~^H P~
                small(2);                                           // T, rank
                bmul(nullptr, Q, 1.0, P, nullptr, nullptr);         // P = P~ T
            }
            PG_HIP(hipGetLastError());
            it += kCheck;
            hipLaunchKernelGGL(k_bred, dim3(C), dim3(256), 0, s, op.ntiles, C, (const double2*)w->p1, norms);
            BlkState bh{};
            PG_HIP(hipMemcpyAsync(nh.data(), norms, sizeof(double2) * C, hipMemcpyDeviceToHost, s));
            PG_HIP(hipMemcpyAsync(&bh, bs, sizeof(bh), hipMemcpyDeviceToHost, s));
            PG_HIP(hipStreamSynchronize(s));
            bool done = bh.stop || bh.rank == 0;
            double worst = 0.0;
            for (int k = 0; k < C; ++k)
                if (tol2[k] < 1e300) worst = std::max(worst, nh[k].x / tol2[k]);
            if (!done) done = worst <= 1.0;
            lowest = std::min(lowest, worst);
            grew = !(worst <= kBlkGrowth * lowest);   // also catches a non-finite norm
            if (done || grew || total + it >= o.max_iter) break;
        }
        total += it;
        if (grew) {
            *handoff = true;
            break;
        }
        PG_TRY(residual());
        PG_TRY(read_state());
        ++restarts;
        if (o.verbose) {
            double wr = 0.0;
            for (int k = 0; k < C; ++k)
                if (w->st_h[k].bnorm > 0) wr = std::max(wr, w->st_h[k].rnorm64 / w->st_h[k].bnorm);
            fprintf(stderr, "[petgem] block COCG: %d iterations, worst true residual %.3e, %.0f ms\n", total, wr,
                    t_all.ms());
            fflush(stderr);
        }
    }
    *block_iters = total;
    if (*handoff) return PETGEM_OK;
    const double t_solve = t_all.ms();
    for (int k = 0; k < C; ++k) {
        petgem_stats* st = stv[k];
        if (!st) continue;
        const ColState& S = w->st_h[k];
        st->iters = total;
        st->block_iters = total;
        st->ir_steps = restarts;
        st->rel_residual = S.bnorm > 0 ? S.rnorm64 / S.bnorm : 0.0;
        st->b_norm = S.bnorm;
        st->x0_rel_residual = 1.0;
        st->t_solve_ms = t_solve;
        st->spmv_shape = 10000 * ch64.kind + 100 * ch64.a + ch64.b;
        st->status = S.outer ? (std::isfinite(S.rnorm64) ? PETGEM_NOT_CONVERGED : PETGEM_NONFINITE) : PETGEM_OK;
        if (st->status != PETGEM_OK && status == PETGEM_OK) status = st->status;
    }
    if (status == PETGEM_NOT_CONVERGED) set_error(std::string("block COCG ") + why + " before rtol");
    if (status == PETGEM_NONFINITE) set_error("non-finite value in the block COCG recurrence");
    return status;
}

}  // namespace

int block_solve(petgem_system* sys, const petgem_source* src, int32_t n_src, const petgem_opts& o,
                const double2* x0, double2* x_out, hipStream_t s, petgem_stats* st) {
    const int n = sys->n_dof, C = n_src;
    const int ntiles = ceil_div(n, kTR);
    const size_t rows = (size_t)ntiles * kTR;
    PG_TRY(ensure_fp32(sys, s));
    PG_TRY(ensure_work(sys->bw, rows, C, C, ntiles));
    BlockWork* w = sys->bw;
    std::vector<double> wmu(C);
    for (int c = 0; c < C; ++c) wmu[c] = 2.0 * kPi * src[c].freq_hz * kMu0;
    int seg_tile[2] = {0, ntiles};
    PG_HIP(hipMemcpyAsync(w->wmu, wmu.data(), sizeof(double) * C, hipMemcpyHostToDevice, s));
    PG_HIP(hipMemcpyAsync(w->seg_tile, seg_tile, sizeof(seg_tile), hipMemcpyHostToDevice, s));
    Op op{};
    op.n = (int)rows;
    op.C = C;
    op.ntiles = ntiles;
    op.nlaunch = ntiles;
    op.nseg = 1;
    op.tile_seg = nullptr;
    op.seg_tile = w->seg_tile;
    op.rp = sys->row_ptr;
    op.col = sys->col;
    op.K32 = sys->K32;
    op.M32 = sys->Ms32;
    op.K64 = sys->K;
    op.M64 = sys->Ms;
    op.Kd = sys->Kd;
    op.Md = sys->Msd;
    op.wmu = w->wmu;
    op.nrow_valid = n;
    if (C <= 4) {   // the sliced-ELLPACK shapes serve up to four columns
        Sell& S = sys->sell32;
        if (!S.ptr || !S.values) PG_TRY(build_sell(S, (int)rows, n, sys->row_ptr, sys->col, sys->K32, sys->Ms32, false, s));
        op.sp = S.ptr;
        op.sw = S.w;
        op.srow = S.row;
        op.scol = S.col;
        op.sK = S.K;
        op.sM = S.M;
    }
    // right-hand sides into the block layout (padding rows stay zero)
    Timer t_rhs;
    hipLaunchKernelGGL(k_fill_z, dim3(ceil_div(rows * C, 256)), dim3(256), 0, s, rows * C, w->B64);
    for (int c = 0; c < C; ++c) PG_TRY(launch_rhs(sys, src[c], w->B64 + c, C, s));
    int flag = 0;
    PG_HIP(hipMemcpyAsync(&flag, sys->dflag, sizeof(int), hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    if (flag) {
        int zero = 0;
        PG_HIP(hipMemcpy(sys->dflag, &zero, sizeof(int), hipMemcpyHostToDevice));
        set_error("source within 1e-9 h of a quadrature point of an element with dsigma != 0");
        return PETGEM_SOURCE_SINGULAR;
    }
    const double trhs = t_rhs.ms();
    hipLaunchKernelGGL(k_fill_z, dim3(ceil_div(rows * C, 256)), dim3(256), 0, s, rows * C, w->X64);
    if (x0)
        hipLaunchKernelGGL(k_cols_in, dim3(ceil_div((size_t)n * C, 256)), dim3(256), 0, s, n, C, (size_t)0,
                           x0, (size_t)n, w->X64);
    std::vector<petgem_stats*> stv(C, nullptr);
    if (st)
        for (int c = 0; c < C; ++c) { stv[c] = st + c; st[c].t_rhs_ms = trhs; }
    if (o.method == PETGEM_BCOCG) {
        bool one_freq = true;
        for (int c = 1; c < C; ++c) one_freq = one_freq && src[c].freq_hz == src[0].freq_hz;
        if (!one_freq || C > kBlkMax || x0 || o.precond != PETGEM_JACOBI) {
            set_error("block COCG: at most 32 sources of one frequency, zero initial guesses, Jacobi");
            return PETGEM_INVALID_ARG;
        }
        bool handoff = false;
        int nblock = 0;
        int rc = bcocg_solve(w, op, sys->nnz, o, s, stv, &handoff, &nblock);
        if (rc != PETGEM_OK && rc != PETGEM_NOT_CONVERGED && rc != PETGEM_NONFINITE) return rc;
        if (handoff) {   // finish as independent mixed COCG columns from the block's iterate
            petgem_opts oc = o;
            oc.method = PETGEM_COCG;
            oc.precision = PETGEM_MIXED;
            oc.max_iter = std::max(1, o.max_iter - nblock);
            rc = mrhs_solve(w, op, sys->nnz, oc, s, stv, true);
            if (rc != PETGEM_OK && rc != PETGEM_NOT_CONVERGED && rc != PETGEM_NONFINITE) return rc;
            for (petgem_stats* p : stv)
                if (p) {
                    p->iters += nblock;
                    p->block_iters = nblock;
                }
        }
        hipLaunchKernelGGL(k_cols_out, dim3(ceil_div((size_t)n * C, 256)), dim3(256), 0, s, n, C, (size_t)0,
                           w->X64, x_out, (size_t)n);
        PG_HIP(hipGetLastError());
        return rc;
    }
    const Ssor* sq = nullptr;
    if (o.precond == PETGEM_SSOR) {
        PG_TRY(ensure_ssor(sys, s));
        sq = &sys->ssor32;
    }
    int rc = mrhs_solve(w, op, sys->nnz, o, s, stv, x0 != nullptr, nullptr, nullptr, sq);
    if (rc != PETGEM_OK && rc != PETGEM_NOT_CONVERGED && rc != PETGEM_NONFINITE) return rc;
    hipLaunchKernelGGL(k_cols_out, dim3(ceil_div((size_t)n * C, 256)), dim3(256), 0, s, n, C, (size_t)0,
                       w->X64, x_out, (size_t)n);
    PG_HIP(hipGetLastError());
    return rc;
}

int batch_solve(petgem_system* const* systems, const petgem_source* src, int32_t n_sys,
                const petgem_opts& o, const void* const* x0, petgem_solution** sols, hipStream_t s,
                petgem_stats* st) {
    // Row offsets of the concatenated block-diagonal operator: every mesh
    // starts on a tile boundary, so each tile belongs to one mesh.
    std::vector<int> row_off(n_sys + 1, 0), seg_tile(n_sys + 1, 0);
    std::vector<int64_t> nnz_off(n_sys + 1, 0);
    for (int k = 0; k < n_sys; ++k) {
        const int nt = ceil_div(systems[k]->n_dof, kTR);
        seg_tile[k + 1] = seg_tile[k] + nt;
        row_off[k + 1] = row_off[k] + nt * kTR;
        nnz_off[k + 1] = nnz_off[k] + systems[k]->nnz;
    }
    const int ntiles = seg_tile[n_sys];
    const size_t rows = (size_t)row_off[n_sys];
    const int64_t nnz = nnz_off[n_sys];
    if (nnz >= (int64_t(1) << 31) || rows >= (size_t(1) << 31)) {
        set_error("uneven batch too large for 32-bit CSR offsets");
        return PETGEM_INVALID_ARG;
    }
    petgem_system* owner = systems[0];
    PG_TRY(ensure_work(owner->bw, rows, 1, n_sys, ntiles));
    BlockWork* w = owner->bw;
    // (re)build the concatenated operator
    if (w->cat_rows < rows || w->cat_nnz < (size_t)nnz) {
        dfree(w->rp); dfree(w->col); dfree(w->K64); dfree(w->M64); dfree(w->K32); dfree(w->M32);
        dfree(w->Kd); dfree(w->Md);
        PG_TRY(dalloc(&w->rp, rows + 1));
        PG_TRY(dalloc(&w->col, (size_t)nnz));
        PG_TRY(dalloc(&w->K64, (size_t)nnz));
        PG_TRY(dalloc(&w->M64, (size_t)nnz));
        PG_TRY(dalloc(&w->K32, (size_t)nnz));
        PG_TRY(dalloc(&w->M32, (size_t)nnz));
        PG_TRY(dalloc(&w->Kd, rows));
        PG_TRY(dalloc(&w->Md, rows));
        w->cat_rows = rows;
        w->cat_nnz = (size_t)nnz;
    }
    std::vector<int> tseg(ntiles);
    std::vector<double> wmu(n_sys);
    for (int k = 0; k < n_sys; ++k) {
        petgem_system* sy = systems[k];
        for (int t = seg_tile[k]; t < seg_tile[k + 1]; ++t) tseg[t] = k;
        wmu[k] = 2.0 * kPi * src[k].freq_hz * kMu0;
        const int n = sy->n_dof;
        hipLaunchKernelGGL(k_cat_rows, dim3(ceil_div(n + 1, 256)), dim3(256), 0, s, n, (int32_t)nnz_off[k],
                           row_off[k], sy->row_ptr, w->rp);
        const int pad = row_off[k + 1] - row_off[k] - n;
        if (pad > 0)
            hipLaunchKernelGGL(k_fill_rp, dim3(ceil_div(pad, 256)), dim3(256), 0, s, pad,
                               (int32_t)nnz_off[k + 1], w->rp + row_off[k] + n + 1);
        hipLaunchKernelGGL(k_cat_cols, dim3(ceil_div(sy->nnz, 256)), dim3(256), 0, s, sy->nnz, row_off[k],
                           sy->col, sy->K, sy->Ms, w->col + nnz_off[k], w->K64 + nnz_off[k],
                           w->M64 + nnz_off[k], w->K32 + nnz_off[k], w->M32 + nnz_off[k]);
        PG_HIP(hipMemcpyAsync(w->Kd + row_off[k], sy->Kd, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        PG_HIP(hipMemcpyAsync(w->Md + row_off[k], sy->Msd, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        if (pad > 0) {
            hipLaunchKernelGGL(k_fill_d, dim3(ceil_div(pad, 256)), dim3(256), 0, s, pad, 1.0, w->Kd + row_off[k] + n);
            hipLaunchKernelGGL(k_fill_d, dim3(ceil_div(pad, 256)), dim3(256), 0, s, pad, 0.0, w->Md + row_off[k] + n);
        }
    }
    PG_HIP(hipGetLastError());
    PG_HIP(hipMemcpyAsync(w->wmu, wmu.data(), sizeof(double) * n_sys, hipMemcpyHostToDevice, s));
    PG_HIP(hipMemcpyAsync(w->seg_tile, seg_tile.data(), sizeof(int) * (n_sys + 1), hipMemcpyHostToDevice, s));
    PG_HIP(hipMemcpyAsync(w->tile_seg, tseg.data(), sizeof(int) * ntiles, hipMemcpyHostToDevice, s));
    Op op{};
    op.n = (int)rows;
    op.C = 1;
    op.ntiles = ntiles;
    op.nlaunch = ntiles;
    op.nseg = n_sys;
    op.tile_seg = w->tile_seg;
    op.seg_tile = w->seg_tile;
    op.rp = w->rp;
    op.col = w->col;
    op.K32 = w->K32;
    op.M32 = w->M32;
    op.K64 = w->K64;
    op.M64 = w->M64;
    op.Kd = w->Kd;
    op.Md = w->Md;
    op.wmu = w->wmu;
    op.nrow_valid = (int)rows;
    PG_TRY(build_sell(w->cat_sell, (int)rows, (int)rows, w->rp, w->col, w->K32, w->M32, true, s));
    op.sp = w->cat_sell.ptr;
    op.sw = w->cat_sell.w;
    op.srow = w->cat_sell.row;
    op.scol = w->cat_sell.col;
    op.sK = w->cat_sell.K;
    op.sM = w->cat_sell.M;
    Timer t_rhs;
    hipLaunchKernelGGL(k_fill_z, dim3(ceil_div(rows, 256)), dim3(256), 0, s, rows, w->B64);
    hipLaunchKernelGGL(k_fill_z, dim3(ceil_div(rows, 256)), dim3(256), 0, s, rows, w->X64);
    bool have_x0 = false;
    std::vector<char> has_x0(n_sys, 0);
    for (int k = 0; x0 && k < n_sys; ++k)
        if (x0[k]) {
            has_x0[k] = 1;
            PG_HIP(hipMemcpyAsync(w->X64 + row_off[k], x0[k], sizeof(double2) * systems[k]->n_dof,
                                  hipMemcpyDeviceToDevice, s));
            have_x0 = true;
        }
    for (int k = 0; k < n_sys; ++k) PG_TRY(launch_rhs(systems[k], src[k], w->B64 + row_off[k], 1, s));
    for (int k = 0; k < n_sys; ++k) {
        int flag = 0;
        PG_HIP(hipMemcpyAsync(&flag, systems[k]->dflag, sizeof(int), hipMemcpyDeviceToHost, s));
        PG_HIP(hipStreamSynchronize(s));
        if (flag) {
            int zero = 0;
            PG_HIP(hipMemcpy(systems[k]->dflag, &zero, sizeof(int), hipMemcpyHostToDevice));
            set_error("source within 1e-9 h of a quadrature point of an element with dsigma != 0 (system " +
                      std::to_string(k) + ")");
            return PETGEM_SOURCE_SINGULAR;
        }
    }
    const double trhs = t_rhs.ms();
    std::vector<petgem_stats*> stv(n_sys, nullptr);
    if (st)
        for (int k = 0; k < n_sys; ++k) { stv[k] = st + k; st[k].t_rhs_ms = trhs; }
    int rc = mrhs_solve(w, op, nnz, o, s, stv, have_x0, &seg_tile, &has_x0);
    if (rc != PETGEM_OK && rc != PETGEM_NOT_CONVERGED && rc != PETGEM_NONFINITE) return rc;
    for (int k = 0; k < n_sys; ++k)
        PG_HIP(hipMemcpyAsync(sols[k]->x, w->X64 + row_off[k], sizeof(double2) * systems[k]->n_dof,
                              hipMemcpyDeviceToDevice, s));
    return rc;
}

}  // namespace petgem
