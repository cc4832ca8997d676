/*
 * petgem.h -- C ABI of the MI355X (gfx950) edge-FEM CSEM secondary-field solver.
 *
 * The library solves, on one GPU, the secondary-field equation of marine
 * controlled-source electromagnetics (Section 2, eq. 6, with the e^{-i w t}
 * sign)
 *
 *     curl curl E_s - i w mu0 sigma E_s = i w mu0 (sigma - sigma_bg) E_p
 *
 * on unstructured tetrahedra with lowest-order Nedelec edge elements
 * (Section 3, eqs. 7-9; Appendix B), E_s = 0 tangentially on the outer
 * boundary (Dirichlet, Section 2), E_p the analytic whole-space dipole field
 * (Appendix A), and returns the total field E_p + E_s at receivers (eq. 8).
 *
 * Conventions
 *   - SI units; time dependence e^{-i w t}; mu0 = 4 pi 1e-7 H/m; w = 2 pi f.
 *   - Complex numbers are interleaved (re, im) pairs of double ("complex128")
 *     or float ("complex64").
 *   - Host pointers are borrowed for the duration of the call only.
 *     Device pointers ("_dev") are caller-owned device memory of the current
 *     HIP device; the library never frees them.
 *   - Handles own their device memory and are released by petgem_free_*.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream). Every
 *     device operation is ordered on it; calls that return host data
 *     synchronise it.
 *   - Every function returning int returns PETGEM_OK (0) or a negative
 *     error code; petgem_last_error() gives a thread-local message. No C++
 *     exception crosses the ABI.
 *   - Unknowns ("DOFs") are the interior edges, ordered by the library; each
 *     DOF is the tangential component of E_s along its edge, directed from
 *     the lower to the higher global node index (Appendix B, eq. B.15).
 */
#ifndef PETGEM_H
#define PETGEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif
#pragma GCC visibility push(default)

/* ---- status codes ------------------------------------------------------ */
#define PETGEM_OK                   0
#define PETGEM_INVALID_ARG         -1  /* null pointer, bad size, bad option   */
#define PETGEM_DEGENERATE_ELEMENT  -2  /* |det J| <= 1e-14 h^3 for an element   */
#define PETGEM_MESH_TOPOLOGY       -3  /* a face shared by more than two tets  */
#define PETGEM_RECEIVER_OUTSIDE    -4  /* a receiver lies in no element        */
#define PETGEM_SOURCE_SINGULAR     -5  /* source within 1e-9 h of a quadrature
                                          point of an element with dsigma != 0 */
#define PETGEM_NOT_CONVERGED       -6  /* max_iter reached; the best iterate is
                                          still returned, stats are filled     */
#define PETGEM_NONFINITE           -7  /* NaN/Inf in the right-hand side or in
                                          the Krylov recurrence                */
#define PETGEM_HIP_ERROR           -8  /* a HIP runtime call failed            */
#define PETGEM_OUT_OF_MEMORY       -9

/* ---- solver options ------------------------------------------------------ */
#define PETGEM_GMRES   0  /* right-Jacobi GMRES(restart), one source at a time */
#define PETGEM_COCG    1  /* multi-source conjugate-orthogonal CG with Jacobi,
                             one sparse matrix pass per iteration for all
                             sources and frequencies                          */
#define PETGEM_JACOBI  0  /* z = D^-1 r, D = diag A                            */
#define PETGEM_SSOR    1  /* multicolour symmetric SOR (the SOR family of the
                             paper's single-process solves, Section 5.3,
                             Table 2): COCG, mixed precision, petgem_solve     */
#define PETGEM_BCOCG   2  /* block COCG: the sources (one frequency, at most
                             32, zero guesses, Jacobi) share one block Krylov
                             space; directions orthonormalised with
                             dependent ones dropped; double precision
                             throughout (precision is ignored), restarted
                             from the true residual. The bilinear form is
                             indefinite, so the block recurrence can lose
                             conjugacy (many nearly dependent sources): the
                             solve then finishes as independent mixed COCG
                             columns from the block's iterate
                             (stats.block_iters)                              */
#define PETGEM_SQMR    3  /* symmetric QMR, the paper's single-process solver
                             (Section 5.3, Table 2), with PETGEM_SSOR only:
                             the COCG recurrence of the preconditioned system
                             plus the quasi-minimal-residual smoothing of its
                             iterate, x_Q = (1 - c^2) x_Q + c^2 x with
                             tau^2 = tau^2 theta^2 c^2, theta = |r| / tau and
                             c^2 = 1 / (1 + theta^2) (|r| in the norm of the
                             inner stop test: the split residual's with more
                             than four sources, the residual's otherwise); each
                             inner solve stops on tau and hands x_Q to the
                             refinement. Mixed precision, like COCG; one more
                             vector (x_Q) is read and written per iteration    */
#define PETGEM_FP64    0  /* every step in double precision                   */
#define PETGEM_MIXED   1  /* complex64 Krylov solves inside a double-precision
                             iterative-refinement loop                         */

typedef struct petgem_system   petgem_system;    /* mesh, matrices, workspaces */
typedef struct petgem_solution petgem_solution;  /* E_s DOFs of n_src sources  */

typedef struct {
    int32_t       n_nodes;
    int32_t       n_tets;
    const double*  xyz;     /* host [n_nodes][3], metres                       */
    const int32_t* tets;    /* host [n_tets][4], 0-based node indices           */
} petgem_mesh;

/* A point electric dipole (Appendix A): moment I*dS along the unit vector
 * dir at pos, frequency freq_hz. */
typedef struct {
    double freq_hz;
    double pos[3];
    double dir[3];
    double moment;          /* I * dS, A*m                                     */
} petgem_source;

typedef struct {
    int32_t method;         /* PETGEM_GMRES, PETGEM_COCG, PETGEM_BCOCG or
                               PETGEM_SQMR                                      */
    int32_t precision;      /* PETGEM_FP64 or PETGEM_MIXED                      */
    int32_t restart;        /* GMRES restart length, 1..64 (default 30)         */
    int32_t max_iter;       /* total Krylov iterations per source               */
    double  rtol;           /* stop when |b - A x|_2 <= rtol |b|_2 (true
                               residual, double precision)                      */
    double  inner_rtol;     /* MIXED: relative tolerance of each inner solve    */
    int32_t use_graph;      /* replay captured HIP graphs for the Krylov loop   */
    int32_t profile;        /* time the sparse-matrix kernels with HIP events   */
    int32_t verbose;        /* print one progress line per refinement step or
                               per 10 GMRES cycles to stderr; 2 (mixed COCG):
                               also one line per column and refinement step    */
    int32_t spmm_shape;     /* COCG: 0 = autotune the complex64 SpMM shape;
                               otherwise that shape, encoded as the
                               spmv_shape statistic (PETGEM_INVALID_ARG if it
                               is not a candidate for this column count, see
                               petgem_spmm_candidates); 40104 / 40108 force
                               the fused single-column step and 50104 / 50108
                               the fused step with one reduction block per
                               mesh, with 4 or 8 slice columns in flight (one
                               column per mesh only; 4010x also needs at most
                               8192 tiles of 256 rows)                         */
    int32_t precond;        /* PETGEM_JACOBI (default) or PETGEM_SSOR. SSOR:
                               the unknowns are coloured so that no two of a
                               colour share a matrix entry (greedy, in the
                               order of the unknowns' global node pairs
                               (lo, hi), smallest colour free among the
                               neighbours); with D = diag A, L / U the entries
                               coupling a row to earlier / later colours,
                               M = (D/omega + L)(D/omega)^-1(D/omega + U), so
                               z = M^-1 r is a forward sweep over the colours
                               and a backward one (complex symmetric: COCG
                               keeps its short recurrence). COCG + MIXED in
                               petgem_solve only (INVALID_ARG otherwise)       */
    double  omega;          /* SSOR relaxation factor, 0 < omega < 2 (1)        */
} petgem_opts;

typedef struct {
    int32_t iters;          /* Krylov iterations (inner ones for MIXED)         */
    int32_t ir_steps;       /* refinement steps (MIXED), restarts (GMRES)       */
    int32_t used_fallback;  /* 1 if the initial guess was rejected for zero     */
    int32_t status;         /* PETGEM_OK or PETGEM_NOT_CONVERGED/NONFINITE      */
    double  rel_residual;   /* final true |b - A x| / |b|                       */
    double  x0_rel_residual;/* |b - A x0| / |b| of the supplied guess (or 1)    */
    double  t_rhs_ms;
    double  t_solve_ms;
    double  spmv_ms;        /* profile: summed duration of sparse-matrix kernels */
    int32_t spmv_launches;  /* profile: number of such launches                  */
    int32_t spmv_shape;     /* COCG: the autotuned complex64 SpMM shape,
                               10000 kind + 100 a + b with kind 0 = CSR column
                               lanes (a lanes per row, b columns per lane),
                               1 = CSR nonzero lanes (a lanes per row, b
                               columns), 2 = sliced ELLPACK (a columns, b
                               slice columns in flight), 3 = sliced ELLPACK
                               with the next b slice columns' indices and
                               values loaded during the current b gathers,
                               4 = the fused step, which one column of one
                               mesh runs whatever shape is tuned (or when
                               shape 3 is chosen): a shape-3 product that
                               also sums q^T D^-1 r and q^T D^-1 q, then one
                               vector kernel applying alpha and beta;
                               5 = the fused step with one reduction block
                               per mesh, which one column per mesh of an
                               uneven batch (or of a mesh with too many
                               tiles for kind 4) runs for a tuned shape;
                               7 = no SpMM: Eisenstat's form of an SSOR
                               block of more than four columns, whose U
                               sweep (with the direction update; a lanes
                               per row, b columns per lane) the profile
                               times instead;
                               GMRES: the lanes per row of the complex128
                               CSR SpMV                                         */
    double  b_norm;         /* |b|_2 of the source's right-hand side            */
    int32_t block_iters;    /* PETGEM_BCOCG: iterations of the block phase; when
                               the block recurrence lost conjugacy (a
                               recursive residual ten times its lowest) the
                               rest of iters ran as independent mixed COCG
                               columns from the block's iterate (0 otherwise) */
    int32_t reserved;
} petgem_stats;

/* Fill *opts with the defaults: GMRES, FP64, restart 30, max_iter 20000,
 * rtol 1e-8, inner_rtol 3e-5, use_graph 1, profile 0, verbose 0, spmm_shape 0,
 * precond PETGEM_JACOBI, omega 1. */
void petgem_default_opts(petgem_opts* opts);

/* ---- assembly (Section 3, eq. 9; Section 4; Appendix B) -----------------
 * Builds the mesh topology on the host (unique edges with the global
 * orientation of eq. B.15, boundary faces and edges, interior DOF numbering,
 * the CSR pattern and the deterministic nnz -> element-entry gather lists),
 * uploads it, and assembles on the GPU the real matrices
 *     K   = sum_e K^e              (eq. B.13, curl-curl)
 *     M_s = sum_e sigma_e M^e      (eq. B.14, mass weighted by sigma)
 * so that A(f) = K - i w mu0 M_s for any frequency.
 *   sigma     host [n_tets] total conductivity, S/m, > 0
 *   sigma_bg  conductivity of the primary field's whole space, > 0
 * Errors: INVALID_ARG, DEGENERATE_ELEMENT, MESH_TOPOLOGY, HIP_ERROR,
 * OUT_OF_MEMORY. On error *out is NULL. */
int petgem_assemble(const petgem_mesh* mesh, const double* sigma, double sigma_bg,
                    void* stream, petgem_system** out);

/* Re-assembles K and M_s on the GPU for new conductivities of the same mesh.
 * sigma_dev: device [n_tets] double. No host work, no allocation. */
int petgem_reassemble(petgem_system* sys, const double* sigma_dev, double sigma_bg,
                      void* stream);

/* ---- background of the primary field --------------------------------------
 * The primary field E_p solves the background problem (Section 2, eqs. 1-6).
 * By default the background is the whole space of conductivity sigma_bg
 * (petgem_assemble) and E_p is the dipole field of Appendix A. With
 * layered = 1 it is two half-spaces meeting at the plane z = z0,
 * sigma_above for z >= z0 (where every source must lie) and sigma_below
 * beneath (a sea over the sea floor), and E_p is the dipole field of that
 * model: the whole-space field of sigma_above plus the wave reflected at the
 * interface above it, the transmitted wave beneath, written as Hankel
 * transforms of the TE / TM interface coefficients and summed by Gauss-
 * Legendre panels on the GPU (one wavefront per evaluation point). The
 * right-hand side then takes dsigma = sigma_e - sigma_b(z) at each
 * quadrature point, so it vanishes wherever the model equals the layers
 * (a mesh whose faces follow the interface confines it to the anomalies).
 * Receivers (petgem_receivers) use the same E_p; petgem_receivers_h refuses a
 * layered background (INVALID_ARG). The setting applies to the following
 * right-hand sides and solves of the system; a solution keeps the background
 * it was solved with. Errors: INVALID_ARG (bad values, or later a source at
 * or below z0). */
typedef struct {
    int32_t layered;        /* 0: whole space sigma_bg; 1: two half-spaces      */
    double  z0;             /* interface height, m                              */
    double  sigma_above;    /* S/m, z >= z0                                     */
    double  sigma_below;    /* S/m, z < z0                                      */
} petgem_background;
int petgem_set_background(petgem_system* sys, const petgem_background* bg);

/* ---- right-hand side (Section 3, eq. 9; Appendix A) ----------------------
 * b_i = i w mu0 sum_e (sigma_e - sigma_bg) sum_q (V_e/4) N_i(x_q) . E_p(x_q)
 * with the 4-point degree-2 rule, for each source, written to
 * b_dev: device complex128 [n_src][n_dof]. */
int petgem_rhs(petgem_system* sys, const petgem_source* src, int32_t n_src,
               void* b_dev, void* stream);

/* The right-hand side of petgem_rhs without any device allocation, for
 * callers that cannot allocate (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc). Same kernels and the same result,
 * bit for bit, as petgem_rhs; their scratch (the element staging and the
 * singular-source flag) is a fixed 48 MiB device array of the library, one
 * copy per GPU, held until the process ends, instead of buffers of the system.
 * Limit: meshes of at most 524,288 elements (INVALID_ARG beyond; use
 * petgem_rhs). The system's device must be current. Every call on one GPU
 * shares the array, so calls that overlap on one GPU (other streams or
 * threads) race; calls ordered on one stream do not. Synchronises `stream`
 * to read the singular-source flag. Errors as petgem_rhs. */
int petgem_rhs_noalloc(petgem_system* sys, const petgem_source* src, int32_t n_src,
                       void* b_dev, void* stream);

/* ---- solve ----------------------------------------------------------------
 * Solves A(f_s) x_s = b_s for every source s (each at its own frequency) to
 * the true relative residual opts->rtol.
 *   x0_dev  optional device complex128 [n_src][n_dof] initial guess (NULL =
 *           zero). Each guess is first scaled by the complex alpha that
 *           minimises |b - alpha A x0|; a guess that is non-finite or still
 *           has |b - A x0| >= |b| is replaced by zero (stats->used_fallback).
 *   *inout  NULL to allocate a new solution, or a solution from an earlier
 *           call on the same system with the same n_src, which is reused.
 *   stats   optional host [n_src].
 * GMRES solves the sources one after another; COCG solves them as one block
 * (all columns in shared launches), except that a large block (n_dof x n_src
 * >= 1e8) whose sources come in contiguous runs of one frequency is solved
 * one run at a time.
 * Returns PETGEM_OK, or NOT_CONVERGED / NONFINITE (the solution then holds
 * the last iterate), or an error. */
int petgem_solve(petgem_system* sys, const petgem_source* src, int32_t n_src,
                 const petgem_opts* opts, const void* x0_dev, void* stream,
                 petgem_solution** inout, petgem_stats* stats);

/* Uneven batch: solves one source on each of n_sys independent systems
 * (different meshes) with the multi-system COCG in mixed precision; the
 * Krylov iterations of all systems run in the same kernel launches, captured
 * once in a HIP graph and replayed until every system has converged.
 *   x0_dev  optional host array of n_sys device pointers, each NULL (zero
 *           guess) or complex128 [n_dof of that system] in the library's DOF
 *           order; every guess is scaled by the alpha minimising
 *           |b - alpha A x0| and one no better than zero (or non-finite) is
 *           replaced by zero for that system alone.
 *   sols[k] as for petgem_solve (n_src = 1), stats host [n_sys]. */
int petgem_solve_many(petgem_system* const* systems, const petgem_source* src,
                      int32_t n_sys, const petgem_opts* opts, const void* const* x0_dev,
                      void* stream, petgem_solution** sols, petgem_stats* stats);

/* ---- receivers (Section 3, eq. 8; Section 2, eq. 4) ----------------------
 * E(x_r) = E_p(x_r) + sum_{i=1..6} N_i(x_r) e_i in the element containing
 * x_r (the lowest element id on faces; all barycentric coordinates
 * >= -1e-12), boundary DOFs being zero.
 *   rx      host [n_rx][3]; located on the host at the first call and cached
 *           while the same coordinates are passed again.
 *   E_dev   device complex128 [n_src][n_rx][3] total field.
 *   Es_dev  optional device complex128 [n_src][n_rx][3] secondary field.
 * Errors: RECEIVER_OUTSIDE, INVALID_ARG, HIP_ERROR. */
int petgem_receivers(const petgem_solution* sol, const double* rx, int32_t n_rx,
                     void* E_dev, void* Es_dev, void* stream);

/* Magnetic field at the receivers (not in the paper, which reports E only):
 * H = curl E / (i w mu0) from Faraday's law of Section 2 (eq. 1, e^{-i w t}),
 * i.e. H_p + curl(sum_i e_i N_i) / (i w mu0) in the receiver's element (the
 * curl of a lowest-order edge field is constant per element; boundary DOFs
 * are zero), H_p = moment (ikr - 1) e^{ikr} / (4 pi r^3) (d x dir) the
 * analytic field of the dipole of Appendix A (d = x - pos). Receivers are
 * located as in petgem_receivers (the same cache).
 *   H_dev   device complex128 [n_src][n_rx][3] total magnetic field, A/m.
 *   Hs_dev  optional device complex128 [n_src][n_rx][3] secondary part.
 * Errors: RECEIVER_OUTSIDE, INVALID_ARG, HIP_ERROR. */
int petgem_receivers_h(const petgem_solution* sol, const double* rx, int32_t n_rx,
                       void* H_dev, void* Hs_dev, void* stream);

/* ---- accessors --------------------------------------------------------- */
int32_t petgem_num_dofs(const petgem_system* sys);
int64_t petgem_nnz(const petgem_system* sys);
int32_t petgem_solution_nsrc(const petgem_solution* sol);
/* Device pointer to the solution DOFs, complex128 [n_src][n_dof] (borrowed). */
const void* petgem_solution_x(const petgem_solution* sol);
/* Copies the solution DOFs into caller device memory x_dev, complex128
 * [n_src][n_dof], ordered on `stream`. */
int petgem_solution_copy(const petgem_solution* sol, void* x_dev, void* stream);
/* Host copies: the global node pair (lo, hi) of every DOF, int32 [n_dof][2];
 * the CSR arrays of K and M_s (row_ptr [n_dof+1], col [nnz], K [nnz],
 * Ms [nnz]). Any output pointer may be NULL. Synchronises the stream. */
int petgem_get_dof_edges(const petgem_system* sys, int32_t* edges);
int petgem_get_csr(const petgem_system* sys, int32_t* row_ptr, int32_t* col,
                   double* K, double* Ms, void* stream);
/* y = A(freq) x for device complex128 vectors of length n_dof, with the
 * kernel the double-precision solver uses. */
int petgem_spmv(petgem_system* sys, double freq, const void* x_dev, void* y_dev,
                void* stream);
/* Host-only preprocessing (no GPU call): the interior-edge numbering and the
 * CSR pattern petgem_assemble would build for this mesh. Call once with the
 * array outputs NULL to get *n_dof and *nnz, then again with
 * dof_edges int32 [n_dof][2] (global node pair lo < hi of each DOF),
 * row_ptr int32 [n_dof+1] and col int32 [nnz]. Errors as petgem_assemble. */
int petgem_mesh_pattern(const petgem_mesh* mesh, int32_t* n_dof, int64_t* nnz,
                        int32_t* dof_edges, int32_t* row_ptr, int32_t* col);
/* Host-only point location (no GPU call): for each point the lowest element
 * id whose barycentric coordinates are all >= -tol, or -1 when the point lies
 * in no element. pts host [n_pts][3], elem host [n_pts]. */
int petgem_locate(const petgem_mesh* mesh, const double* pts, int32_t n_pts, double tol,
                  int32_t* elem);
/* Autotuner choices of a system: lanes per row of the double-precision CSR
 * SpMV (4, 8 or 16; 0 before the first solve) and the measured per-launch
 * times of the three variants in ms (host float [3], may be NULL). */
int petgem_tuning(const petgem_system* sys, int32_t* spmv_group, float* spmv_ms);
/* Seconds spent in the host preprocessing of the last petgem_assemble. */
double petgem_setup_seconds(const petgem_system* sys);
/* The multicolour SSOR preconditioner of PETGEM_SSOR (see petgem_opts):
 * petgem_ssor_colors writes the colour of every DOF (host int32 [n_dof],
 * library DOF order) and returns the number of colours (builds the colouring
 * if needed; synchronises `stream`). petgem_ssor_apply computes z = M^-1 r
 * for one complex64 column at frequency freq: r_dev, z_dev device complex64
 * [n_dof], distinct; synchronises `stream`. */
int32_t petgem_ssor_colors(petgem_system* sys, int32_t* colors, void* stream);
int petgem_ssor_apply(petgem_system* sys, double freq, double omega, const void* r_dev, void* z_dev,
                      void* stream);
/* Measurement behind the uneven batch's design (graph-replayed kernels rather
 * than one persistent kernel): the time per round of `rounds` phase
 * separations, mode 0 = a kernel boundary inside a captured HIP graph
 * (rounds launches of a one-word-per-block kernel), mode 1 = a grid-wide
 * barrier inside one cooperative kernel of as many 256-thread blocks as can be
 * resident (*blocks receives that count). Synchronises `stream`. Errors:
 * INVALID_ARG (rounds outside 1..100000, mode), HIP_ERROR (the runtime
 * refused the cooperative launch). */
int petgem_sync_probe(int32_t rounds, int32_t mode, int32_t* blocks, float* us_per_round, void* stream);
/* Host-only: the complex64 SpMM shapes the autotuner times for n_cols
 * columns (sliced != 0: with the sliced-ELLPACK copy, which one mesh has for
 * up to four columns), as petgem_opts.spmm_shape codes. Writes at most cap
 * codes to shapes (host int32, may be NULL when cap is 0) and returns how
 * many there are, or PETGEM_INVALID_ARG. */
int32_t petgem_spmm_candidates(int32_t n_cols, int32_t sliced, int32_t* shapes, int32_t cap);

/* ---- learned initial guess (not in the paper) -------------------------------
 * A small 3D U-Net on a 32^3 voxel grid covering the mesh's bounding box
 * (cubic cells of side max extent / 32) predicts the secondary field at the
 * voxel centres, scaled by 1 / (g |b|); it is interpolated trilinearly to the
 * edge midpoints and projected on the edge tangents to give an initial guess.
 * Input tensor X: bf16 [B][32^3][16] (z-major voxels, channels last):
 * log10 sigma of the containing element, (x - x_s)/L, (y - y_s)/L,
 * (z - z_s)/L with L = half the box side, log10 f, then zeros. Output tensor
 * Y: float [B][32^3][16], channels 0..5 = Re Ex, Im Ex, Re Ey, Im Ey, Re Ez,
 * Im Ez (scaled). Targets T: float [B][32^3][6]. Parameters: float, layer by
 * layer W[27][Cin][Cout] (tap = 9 (dz+1) + 3 (dy+1) + (dx+1)) then b[Cout],
 * for (Cin, Cout) = (16,16), (16,32), (32,64), (64,64), (96,32), (48,16),
 * (16,16). Loss: mean squared error over the 6 used channels. */
typedef struct petgem_net petgem_net;
int petgem_net_create(int32_t batch_max, uint64_t seed, petgem_net** out);
int64_t petgem_net_num_params(const petgem_net* net);
int petgem_net_get_params(const petgem_net* net, float* host);
int petgem_net_set_params(petgem_net* net, const float* host);
/* y_dev = network(x_dev) for `batch` samples (device pointers). */
int petgem_net_forward(petgem_net* net, const void* x_dev, int32_t batch, void* y_dev, void* stream);
/* Loss and its gradient with respect to every parameter (host copy if
 * grad_host is not NULL); the parameters are not changed. */
int petgem_net_loss_grad(petgem_net* net, const void* x_dev, const void* t_dev, int32_t batch,
                         void* stream, double* loss, float* grad_host);
/* One Adam step (beta 0.9, 0.999, eps 1e-8) on the batch's loss. */
int petgem_net_train_step(petgem_net* net, const void* x_dev, const void* t_dev, int32_t batch,
                          float lr, void* stream, double* loss);
/* Network inputs of `batch` (conductivity model, source) pairs on a system's
 * mesh: sigma_dev device double [batch][n_tets], or NULL for the system's
 * current conductivities; x_dev as X above. */
int petgem_voxelize(petgem_system* sys, const double* sigma_dev, const petgem_source* src,
                    int32_t batch, void* x_dev, void* stream);
/* Training targets from a solution: E_s at the voxel centres divided by
 * scale[k] (host double [n_src]), t_dev as T above. */
int petgem_vox_targets(const petgem_solution* sol, const double* scale, void* t_dev, void* stream);
/* Initial guess for petgem_solve: computes |b| of every source, runs the
 * network on the system's current conductivities and writes x0_dev
 * (complex128 [batch][n_dof]) = g |b| (predicted field at the edge
 * midpoint . edge tangent). bnorm_out (host [batch], may be NULL) receives
 * |b|. */
int petgem_learned_x0(petgem_system* sys, petgem_net* net, const petgem_source* src, int32_t batch,
                      double g, void* x0_dev, double* bnorm_out, void* stream);
/* petgem_learned_x0 for n_sys systems with one source each, run as one
 * network batch (n_sys <= the network's batch_max): sample k is system k's
 * conductivities on its own voxel grid with src[k]. x0_dev[k] is caller-owned
 * device complex128 [n_dof of system k]; bnorm_out (host [n_sys], may be
 * NULL) receives |b| of every system. Each guess equals what
 * petgem_learned_x0 gives for that system and source alone. */
int petgem_learned_x0_many(petgem_system* const* systems, petgem_net* net, const petgem_source* src,
                           int32_t n_sys, double g, void* const* x0_dev, double* bnorm_out, void* stream);
void petgem_net_free(petgem_net* net);

void petgem_free_system(petgem_system* sys);
void petgem_free_solution(petgem_solution* sol);
const char* petgem_last_error(void);

#pragma GCC visibility pop
#ifdef __cplusplus
}
#endif
#endif /* PETGEM_H */
