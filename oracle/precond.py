"""Oracle: the multicolour SSOR preconditioner, written out plainly.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper's single-process solves precondition SQMR with SOR (Section 5.3,
Table 2). Its symmetric form for a complex-symmetric A, made parallel by a
colouring of the unknowns, is defined here:

* Colouring: the unknowns in increasing order of their global node pair
  (lo, hi) -- the oracle's own DOF order -- each taking the smallest colour
  that none of its matrix neighbours already has (greedy).
* With D = diag A and L (U) the entries of A that couple a row to a row of an
  earlier (later) colour -- no two rows of one colour are coupled, so
  A = D + L + U with U = L^T --
      M = (D / omega + L) (D / omega)^-1 (D / omega + U)
  (the constant (2 - omega) / omega of the textbook SSOR left out).
* z = M^-1 r: the forward sweep (D / omega + L) y = r taken colour by colour
  in increasing order, then the backward sweep (D / omega + U) z = (D / omega) y
  in decreasing order.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def greedy_colors(A: sp.csr_matrix) -> np.ndarray:
    """Colour of every row, greedy in row order (smallest colour not taken by
    an already coloured neighbour)."""
    A = A.tocsr()
    n = A.shape[0]
    color = np.full(n, -1, dtype=np.int64)
    for i in range(n):
        taken = set(int(c) for c in color[A.indices[A.indptr[i]:A.indptr[i + 1]]] if c >= 0)
        c = 0
        while c in taken:
            c += 1
        color[i] = c
    return color


def split(A: sp.csr_matrix, color: np.ndarray):
    """(D, L, U): the diagonal and the parts of A to earlier / later colours."""
    A = A.tocoo()
    lo = color[A.col] < color[A.row]
    hi = color[A.col] > color[A.row]
    n = A.shape[0]
    L = sp.csr_matrix((A.data[lo], (A.row[lo], A.col[lo])), shape=(n, n))
    U = sp.csr_matrix((A.data[hi], (A.row[hi], A.col[hi])), shape=(n, n))
    return A.tocsr().diagonal(), L, U


def ssor_apply(A: sp.csr_matrix, color: np.ndarray, omega: float, r: np.ndarray) -> np.ndarray:
    """z = M^-1 r by the two colour sweeps (complex128)."""
    d, L, U = split(A, color)
    r = np.asarray(r, dtype=np.complex128)
    y = np.zeros_like(r)
    for c in range(int(color.max()) + 1):
        rows = np.flatnonzero(color == c)
        y[rows] = omega * (r[rows] - L[rows] @ y) / d[rows]
    z = y.copy()
    for c in range(int(color.max()), -1, -1):
        rows = np.flatnonzero(color == c)
        z[rows] = y[rows] - omega * (U[rows] @ z) / d[rows]
    return z


def ssor_matrix(A: sp.csr_matrix, color: np.ndarray, omega: float) -> sp.csr_matrix:
    """M itself, as a sparse product (for pins)."""
    d, L, U = split(A, color)
    Dw = sp.diags(d / omega)
    return ((Dw + L) @ sp.diags(omega / d) @ (Dw + U)).tocsr()


def cocg(A: sp.csr_matrix, b: np.ndarray, apply_m, rtol: float = 1e-10, max_iter: int = 20000):
    """Preconditioned conjugate orthogonal CG (bilinear u^T v, the complex
    symmetric analogue of CG) to |b - A x| <= rtol |b|. Returns (x, its)."""
    x = np.zeros_like(b)
    r = b.copy()
    z = apply_m(r)
    p = z.copy()
    rho = r @ z
    bn = np.linalg.norm(b)
    for it in range(1, max_iter + 1):
        q = A @ p
        alpha = rho / (p @ q)
        x = x + alpha * p
        r = r - alpha * q
        if np.linalg.norm(r) <= rtol * bn:
            return x, it
        z = apply_m(r)
        rho_new = r @ z
        p = z + (rho_new / rho) * p
        rho = rho_new
    return x, max_iter
