"""Oracle: solves of the assembled secondary-field system and the end-to-end
receiver response.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper solves with PETSc GMRES (Section 5.1), SQMR with SOR (Section 5.3)
or MUMPS (Section 5.2). The oracle reaches the same discrete solution by the
most direct route available at each size: a dense LU solve, SciPy's sparse LU,
or a plain right-Jacobi-preconditioned restarted GMRES (modified Gram-Schmidt,
Givens rotations) driven to a true relative residual of 1e-12, tighter than
the 1e-8 of the GPU solve so that the oracle's own error stays far below the
1e-6 receiver budget.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import scipy.linalg as sla
from scipy.linalg import blas
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem


class RowBlockMatvec:
    """y = A x by row blocks on a thread pool (SciPy's CSR product releases
    the interpreter lock). Each row's sum is the same as in A @ x, so the
    result is bitwise that of the one-thread product; only the wall time
    changes."""

    def __init__(self, A: sp.csr_matrix, threads: int | None = None):
        self.threads = threads or int(os.environ.get("ORACLE_THREADS", len(os.sched_getaffinity(0))))
        n = A.shape[0]
        self.A = A
        if self.threads <= 1 or A.nnz < 1_000_000:
            self.blocks = None
            return
        cuts = np.linspace(0, n, self.threads + 1).astype(np.int64)
        self.blocks = [A[cuts[i]:cuts[i + 1]] for i in range(self.threads)]
        self.pool = ThreadPoolExecutor(self.threads)

    def __matmul__(self, x):
        if self.blocks is None:
            return self.A @ x
        return np.concatenate(list(self.pool.map(lambda B: B @ x, self.blocks)))


def gmres(A: sp.csr_matrix, b: np.ndarray, rtol: float = 1e-12, restart: int = 60,
          max_iter: int = 200000, x0=None, progress: int = 0):
    """Restarted GMRES on A D^{-1} y = b, x = D^{-1} y with D = diag(A).
    Stops when the true residual |b - A x| / |b| <= rtol (checked at every
    restart). Returns (x, iterations, true relative residual).
    Gram-Schmidt is the modified one; its updates are in-place BLAS axpy
    (w <- w - h v), and the products run by row blocks on threads
    (`RowBlockMatvec`): neither changes what is computed."""
    n = len(b)
    dinv = 1.0 / A.diagonal()
    A = RowBlockMatvec(A)
    x = np.zeros(n, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return np.zeros(n, dtype=np.complex128), 0, 0.0
    it = 0
    while True:
        r = b - A @ x
        rn = np.linalg.norm(r)
        if progress:
            print(f"oracle gmres: {it} iterations, true relative residual {rn / bn:.3e}", flush=True)
        if rn <= rtol * bn or it >= max_iter:
            return x, it, rn / bn
        V = np.zeros((restart + 1, n), dtype=np.complex128)
        H = np.zeros((restart + 1, restart), dtype=np.complex128)
        cs = np.zeros(restart, dtype=np.complex128)
        sn = np.zeros(restart, dtype=np.complex128)
        g = np.zeros(restart + 1, dtype=np.complex128)
        V[0] = r / rn
        g[0] = rn
        m = 0
        for j in range(restart):
            w = A @ (dinv * V[j])
            for i in range(j + 1):
                H[i, j] = np.vdot(V[i], w)
                w = blas.zaxpy(V[i], w, a=-H[i, j])
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0.0:
                V[j + 1] = w / H[j + 1, j]
            # rotation i acts on rows (i, i+1) as [[conj(c), conj(s)], [-s, c]]
            for i in range(j):
                t = np.conj(cs[i]) * H[i, j] + np.conj(sn[i]) * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.sqrt(abs(H[j, j]) ** 2 + abs(H[j + 1, j]) ** 2)
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = np.conj(cs[j]) * g[j]
            m = j + 1
            it += 1
            if abs(g[j + 1]) <= 0.1 * rtol * bn or it >= max_iter:
                break
        y = sla.solve_triangular(H[:m, :m], g[:m])
        x = x + dinv * (V[:m].T @ y)


def _one_blas_thread():
    """One BLAS thread for the enclosed calls (arithmetic unchanged)."""
    try:
        from threadpoolctl import threadpool_limits
        return threadpool_limits(limits=1, user_api="blas")
    except ImportError:   # pragma: no cover - the limit is only a speed matter
        import contextlib
        return contextlib.nullcontext()


def solve_system(A: sp.csr_matrix, b: np.ndarray, rtol: float = 1e-12, progress: int = 0):
    """Dense LU up to 6000 unknowns, sparse LU up to 60000, GMRES above.
    Returns (x, true relative residual, method)."""
    n = A.shape[0]
    bn = np.linalg.norm(b)
    if n <= 6000:
        x = np.linalg.solve(A.toarray(), b)
        method = "dense"
    elif n <= 60000:
        # SuperLU's dense kernels are small: one BLAS thread (several spin
        # against each other and slow the factorisation down many times
        # whenever other work shares the cores)
        with _one_blas_thread():
            x = spla.spsolve(A.tocsc(), b)
        method = "splu"
    else:
        with _one_blas_thread():   # the row-block products have their own threads
            x, _, _ = gmres(A, b, rtol=rtol, progress=progress)
        method = "gmres"
    res = np.linalg.norm(b - A @ x) / bn if bn > 0 else 0.0
    return x, res, method


def forward(model, src_index: int = 0, sys_=None, rtol: float = 1e-12, progress: int = 0):
    """End-to-end oracle response of one source: assemble, right-hand side,
    solve, total field at the receivers. Returns a dict."""
    xyz, tets = model.xyz, model.tets
    if sys_ is None:
        sys_ = fem.assemble(xyz, tets, model.sigma)
    s = model.sources[src_index]
    A = fem.system_matrix(sys_, s.freq)
    layers = getattr(model, "layers", None)
    if layers is None:
        b = fem.rhs(xyz, tets, model.sigma, model.sigma_bg, sys_.topo, s.pos, s.dir,
                    s.freq, s.moment)
    else:
        b = fem.rhs_layered(xyz, tets, model.sigma, layers, sys_.topo, s.pos, s.dir, s.freq, s.moment)
    x, res, method = solve_system(A, b, rtol, progress)
    if layers is None:
        E = fem.receivers_total(xyz, tets, sys_.topo, x, model.receivers, s.pos, s.dir,
                                s.freq, model.sigma_bg, s.moment)
    else:
        E = fem.receivers_total_layered(xyz, tets, sys_.topo, x, model.receivers, s.pos, s.dir, s.freq,
                                        layers, s.moment)
    Es = fem.interpolate(xyz, tets, sys_.topo, x, model.receivers)
    return dict(x=x, b=b, A=A, E=E, Es=Es, residual=res, method=method, sys=sys_)
