"""High-order reference quadrature on tetrahedra for the oracle's pins.

A conical (Duffy) product rule: Gauss-Legendre points (u, v, w) on [0,1]^3
mapped by xi1 = u, xi2 = v (1-u), xi3 = w (1-u)(1-v) with Jacobian
(1-u)^2 (1-v). With q points per direction it integrates polynomials of
degree <= 2q - 3 exactly. It shares nothing with the 4-point rule of the
method and is used only to check things independently of it.
"""
import numpy as np


def duffy_rule(q: int = 5):
    """Barycentric points [P][4] and weights [P] summing to 1 (fraction of V)."""
    g, w = np.polynomial.legendre.leggauss(q)
    g = 0.5 * (g + 1.0)
    w = 0.5 * w
    U, Vv, W = np.meshgrid(g, g, g, indexing="ij")
    WU, WV, WW = np.meshgrid(w, w, w, indexing="ij")
    xi1 = U
    xi2 = Vv * (1 - U)
    xi3 = W * (1 - U) * (1 - Vv)
    jac = (1 - U) ** 2 * (1 - Vv)
    wt = (WU * WV * WW * jac).ravel() * 6.0      # reference volume is 1/6
    lam = np.stack([1 - xi1 - xi2 - xi3, xi1, xi2, xi3], axis=-1).reshape(-1, 4)
    return lam, wt


def tet_points(X: np.ndarray, lam: np.ndarray) -> np.ndarray:
    """Physical points [T][P][3] of barycentric points lam [P][4] in tets X [T][4][3]."""
    return np.einsum("pv,tvk->tpk", lam, X)


def tet_volumes(X: np.ndarray) -> np.ndarray:
    d1, d2, d3 = X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]
    return np.abs(np.einsum("tk,tk->t", d1, np.cross(d2, d3))) / 6.0


def barycentric_by_solve(X: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """lambda at points by solving [x; 1] = [X^T; 1] lambda per element
    (no gradient formula involved). X [T][4][3], pts [T][P][3] -> [T][P][4]."""
    T = len(X)
    Mx = np.ones((T, 4, 4))
    Mx[:, :3, :] = np.transpose(X, (0, 2, 1))
    rhs = np.ones(pts.shape[:2] + (4,))
    rhs[..., :3] = pts
    return np.linalg.solve(Mx[:, None], rhs[..., None])[..., 0]
