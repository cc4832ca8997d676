"""Oracle: lowest-order Nedelec edge elements on tetrahedra, assembly of the
secondary-field system, right-hand side and receiver interpolation.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``). Plain NumPy/SciPy in
float64 / complex128; no blocking, fusion or reordering beyond the
definitions below.

Conventions (with the readings listed in the design notes):

* Local edges (Appendix B, eqs. B.1-B.6, figure of the edge element), with the
  vertices numbered 1..4 there and 0..3 here: e1 (1,2), e2 (1,3), e3 (1,4),
  e4 (2,3), e5 (4,2), e6 (3,4).
* Global orientation of an edge: from the lower to the higher global node
  index; the local sign is s_i = sign(g(i2) - g(i1)) (Appendix B, eq. B.15,
  read as +-1 over global node indices).
* Basis: N_i = s_i l_i (lambda_a grad lambda_b - lambda_b grad lambda_a)
  (Appendix B, eqs. B.1-B.12, with the edge length l_i); its degree of freedom
  is the tangential component of E along the global edge direction (Section 3,
  text before eq. 8).
* Element matrices (Appendix B, eqs. B.13, B.14):
  K_ij = int curl N_i . curl N_j dV,  M_ij = int N_i . N_j dV.
* Secondary-field system (Section 2, eq. 6 and Section 3, eqs. 7 and 9) with
  the e^{-i omega t} sign and mu0 restored:
  (K - i omega mu0 M_sigma) e = b,   M_sigma = sum_e sigma_e M^e,
  b_i = i omega mu0 sum_e dsigma_e int N_i . E_p dV,  dsigma = sigma - sigma_bg.
* Homogeneous Dirichlet condition (Section 2, after eq. 6) by eliminating every
  edge of a boundary face; the unknowns are the interior edges.
* Right-hand-side quadrature: the 4-point degree-2 symmetric rule on the
  tetrahedron (the paper says only that R^e needs numerical integration).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .primary import MU0, dipole_field, dipole_magnetic_field

LOCAL_EDGES = np.array([(0, 1), (0, 2), (0, 3), (1, 2), (3, 1), (2, 3)], dtype=np.int64)
FACES = np.array([(1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2)], dtype=np.int64)

_QA = (5.0 + 3.0 * np.sqrt(5.0)) / 20.0
_QB = (5.0 - np.sqrt(5.0)) / 20.0
# Barycentric points (rows) of the 4-point rule; each weight is V/4.
QUAD4 = np.array([[_QA, _QB, _QB, _QB], [_QB, _QA, _QB, _QB],
                  [_QB, _QB, _QA, _QB], [_QB, _QB, _QB, _QA]])


@dataclass
class Topology:
    edge_nodes: np.ndarray     # int64 [E][2], lo < hi global node index
    elem_edge: np.ndarray      # int64 [T][6] global edge of each local edge
    elem_sign: np.ndarray      # float64 [T][6] s_i = +-1
    boundary_edge: np.ndarray  # bool [E]
    dof_of_edge: np.ndarray    # int64 [E] interior numbering, -1 on the boundary
    n_dof: int
    boundary_node: np.ndarray  # bool [N]


def topology(xyz: np.ndarray, tets: np.ndarray) -> Topology:
    """Unique edges with global orientation and local signs (Appendix B,
    eq. B.15); boundary faces are faces of exactly one tetrahedron, boundary
    edges the edges of boundary faces (Section 2, Dirichlet condition)."""
    tets = np.asarray(tets, dtype=np.int64)
    n_nodes = len(xyz)
    a = tets[:, LOCAL_EDGES[:, 0]]
    b = tets[:, LOCAL_EDGES[:, 1]]
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    key = lo * n_nodes + hi
    uniq, inv = np.unique(key.ravel(), return_inverse=True)
    edge_nodes = np.stack([uniq // n_nodes, uniq % n_nodes], axis=1)
    elem_edge = inv.reshape(-1, 6)
    elem_sign = np.where(b > a, 1.0, -1.0)

    f = np.sort(tets[:, FACES], axis=2).reshape(-1, 3)
    fkey = (f[:, 0] * n_nodes + f[:, 1]) * n_nodes + f[:, 2]
    fu, fcount = np.unique(fkey, return_counts=True)
    if np.any(fcount > 2):
        raise ValueError("mesh topology: a face is shared by more than two elements")
    bf = fu[fcount == 1]
    bfn = np.stack([bf // (n_nodes * n_nodes), (bf // n_nodes) % n_nodes, bf % n_nodes], 1)
    boundary_edge = np.zeros(len(uniq), dtype=bool)
    for p, q in ((0, 1), (0, 2), (1, 2)):
        k = bfn[:, p] * n_nodes + bfn[:, q]
        boundary_edge[np.searchsorted(uniq, k)] = True
    boundary_node = np.zeros(n_nodes, dtype=bool)
    boundary_node[bfn.ravel()] = True
    dof = np.full(len(uniq), -1, dtype=np.int64)
    interior = np.flatnonzero(~boundary_edge)
    dof[interior] = np.arange(len(interior))
    return Topology(edge_nodes, elem_edge, elem_sign, boundary_edge, dof,
                    len(interior), boundary_node)


def geometry(xyz: np.ndarray, tets: np.ndarray):
    """Volumes V = |det J| / 6 and barycentric gradients grad lambda [T][4][3]
    (Appendix B, gradient expansion): with J = [x1-x0, x2-x0, x3-x0] as
    columns, grad lambda_{1,2,3} are the rows of J^{-1} and
    grad lambda_0 = -sum of the others."""
    X = np.asarray(xyz, dtype=np.float64)[np.asarray(tets)]
    J = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
    det = np.linalg.det(J)
    vol = np.abs(det) / 6.0
    Jinv = np.linalg.inv(J)
    g = np.empty((len(X), 4, 3))
    g[:, 1:, :] = Jinv
    g[:, 0, :] = -Jinv.sum(axis=1)
    return vol, g, X


def edge_lengths(X: np.ndarray) -> np.ndarray:
    d = X[:, LOCAL_EDGES[:, 1]] - X[:, LOCAL_EDGES[:, 0]]
    return np.sqrt(np.sum(d * d, axis=2))


def element_matrices(xyz: np.ndarray, tets: np.ndarray, sign: np.ndarray):
    """K^e and M^e [T][6][6] (Appendix B, eqs. B.13 and B.14).

    K: curl N_i = 2 s_i l_i grad lambda_a x grad lambda_b is constant, so
    K_ij = V curl N_i . curl N_j.
    M: expanding N_i . N_j and integrating with
    int lambda_p lambda_q dV = V (1 + delta_pq) / 20 gives
    M_ij = s_i s_j l_i l_j [I_ac g_bd - I_ad g_bc - I_bc g_ad + I_bd g_ac],
    g_pq = grad lambda_p . grad lambda_q, for edges i = (a, b), j = (c, d)."""
    vol, g, X = geometry(xyz, tets)
    if np.any(vol <= 0.0):
        raise ValueError("degenerate element")
    ell = edge_lengths(X)
    ea, eb = LOCAL_EDGES[:, 0], LOCAL_EDGES[:, 1]
    curl = 2.0 * (sign * ell)[:, :, None] * np.cross(g[:, ea], g[:, eb])
    K = vol[:, None, None] * np.einsum("tik,tjk->tij", curl, curl)
    G = np.einsum("tpk,tqk->tpq", g, g)
    I = (np.ones((4, 4)) + np.eye(4)) / 20.0
    M = np.empty_like(K)
    for i in range(6):
        a, b = ea[i], eb[i]
        for j in range(6):
            c, d = ea[j], eb[j]
            M[:, i, j] = (I[a, c] * G[:, b, d] - I[a, d] * G[:, b, c]
                          - I[b, c] * G[:, a, d] + I[b, d] * G[:, a, c])
    sl = sign * ell
    M *= vol[:, None, None] * sl[:, :, None] * sl[:, None, :]
    return K, M


def basis_at(g: np.ndarray, sign: np.ndarray, ell: np.ndarray, lam: np.ndarray) -> np.ndarray:
    """N_i at barycentric points: g [T][4][3], lam [T][Q][4] -> [T][Q][6][3]."""
    ea, eb = LOCAL_EDGES[:, 0], LOCAL_EDGES[:, 1]
    la, lb = lam[:, :, ea], lam[:, :, eb]                       # [T][Q][6]
    ga, gb = g[:, None, ea, :], g[:, None, eb, :]               # [T][1][6][3]
    w = la[..., None] * gb - lb[..., None] * ga
    return (sign * ell)[:, None, :, None] * w


@dataclass
class System:
    topo: Topology
    K: sp.csr_matrix           # interior-edge curl-curl matrix (real)
    Ms: sp.csr_matrix          # interior-edge sigma-weighted mass matrix (real)


def assemble(xyz, tets, sigma, topo: Topology | None = None, full: bool = False) -> System:
    """Global K and M_sigma = sum_e sigma_e M^e from the element matrices
    (Section 3, eq. 9; Section 4: each element adds its contribution), as COO
    with duplicates summed. ``full`` keeps the boundary edges (numbered by
    global edge index) for the whole-space identities used as pins."""
    topo = topo or topology(xyz, tets)
    Ke, Me = element_matrices(xyz, tets, topo.elem_sign)
    Me = Me * np.asarray(sigma, dtype=np.float64)[:, None, None]
    idx = topo.elem_edge if full else topo.dof_of_edge[topo.elem_edge]
    n = len(topo.edge_nodes) if full else topo.n_dof
    r = np.repeat(idx[:, :, None], 6, axis=2)
    c = np.repeat(idx[:, None, :], 6, axis=1)
    keep = (r >= 0) & (c >= 0)
    K = sp.coo_matrix((Ke[keep], (r[keep], c[keep])), shape=(n, n)).tocsr()
    M = sp.coo_matrix((Me[keep], (r[keep], c[keep])), shape=(n, n)).tocsr()
    K.sum_duplicates()
    M.sum_duplicates()
    return System(topo, K, M)


def system_matrix(sys_: System, freq: float) -> sp.csr_matrix:
    """A = K - i omega mu0 M_sigma."""
    omega = 2.0 * np.pi * freq
    return (sys_.K.astype(np.complex128) - 1j * omega * MU0 * sys_.Ms).tocsr()


def rhs(xyz, tets, sigma, sigma_bg, topo: Topology, src_pos, src_dir, freq,
        moment=1.0, field=None) -> np.ndarray:
    """b_i = i omega mu0 sum_e dsigma_e sum_q w_q N_i(x_q) . E_p(x_q) over the
    elements with dsigma_e != 0 (Section 3, eq. 9; Appendix A for E_p).
    ``field`` (points [..][3] -> complex [..][3]) replaces E_p when given
    (a test hook: a field in the edge-element space has a closed-form
    right-hand side)."""
    sigma = np.asarray(sigma, dtype=np.float64)
    dsig = sigma - sigma_bg
    sel = np.flatnonzero(dsig != 0.0)
    b = np.zeros(topo.n_dof, dtype=np.complex128)
    if len(sel) == 0:
        return b
    t = np.asarray(tets)[sel]
    vol, g, X = geometry(xyz, t)
    ell = edge_lengths(X)
    sign = topo.elem_sign[sel]
    lam = np.broadcast_to(QUAD4, (len(sel), 4, 4))
    xq = np.einsum("tqv,tvk->tqk", lam, X)
    if field is None:
        Ep = dipole_field(xq, src_pos, src_dir, freq, sigma_bg, moment)   # [T][4][3]
    else:
        Ep = np.asarray(field(xq), dtype=np.complex128)
    N = basis_at(g, sign, ell, lam)                                        # [T][4][6][3]
    Re = (vol / 4.0)[:, None] * np.einsum("tqik,tqk->ti", N, Ep)           # [T][6]
    omega = 2.0 * np.pi * freq
    contrib = 1j * omega * MU0 * dsig[sel][:, None] * Re
    dof = topo.dof_of_edge[topo.elem_edge[sel]]
    keep = dof >= 0
    np.add.at(b, dof[keep], contrib[keep])
    return b


def background_sigma(z, layers) -> np.ndarray:
    """sigma of the layered background at heights z: layers = (z0,
    sigma_above, sigma_below); a point on z0 counts as above."""
    z0, s_up, s_dn = layers
    return np.where(np.asarray(z) >= z0, s_up, s_dn)


def rhs_layered(xyz, tets, sigma, layers, topo: Topology, src_pos, src_dir, freq,
                moment=1.0) -> np.ndarray:
    """Eq. 9 with a background of two half-spaces: the primary field is the
    layered one (``oracle.layered``) and dsigma = sigma_e - sigma_b(x_q) is
    taken at each quadrature point:
    b_i = i omega mu0 sum_e sum_q (V_e/4) dsigma_eq N_i(x_q) . E_p(x_q)."""
    from .layered import layered_dipole_field
    sigma = np.asarray(sigma, dtype=np.float64)
    t_all = np.asarray(tets)
    X_all = np.asarray(xyz, dtype=np.float64)[t_all]
    xq_all = np.einsum("qv,tvk->tqk", QUAD4, X_all)                       # [T][4][3]
    dsig = sigma[:, None] - background_sigma(xq_all[..., 2], layers)      # [T][4]
    sel = np.flatnonzero(np.any(dsig != 0.0, axis=1))
    b = np.zeros(topo.n_dof, dtype=np.complex128)
    if len(sel) == 0:
        return b
    vol, g, X = geometry(xyz, t_all[sel])
    ell = edge_lengths(X)
    sign = topo.elem_sign[sel]
    lam = np.broadcast_to(QUAD4, (len(sel), 4, 4))
    xq = xq_all[sel]
    Ep = layered_dipole_field(xq, src_pos, src_dir, freq, layers[1], layers[2], layers[0], moment)
    N = basis_at(g, sign, ell, lam)                                        # [T][4][6][3]
    Re = (vol / 4.0)[:, None] * np.einsum("tq,tqik,tqk->ti", dsig[sel], N, Ep)
    omega = 2.0 * np.pi * freq
    contrib = 1j * omega * MU0 * Re
    dof = topo.dof_of_edge[topo.elem_edge[sel]]
    keep = dof >= 0
    np.add.at(b, dof[keep], contrib[keep])
    return b


def receivers_total_layered(xyz, tets, topo, e_dof, points, src_pos, src_dir, freq, layers,
                            moment=1.0) -> np.ndarray:
    """Total field E = E_p (layered) + E_s at the receivers (eq. 4)."""
    from .layered import layered_dipole_field
    return (layered_dipole_field(points, src_pos, src_dir, freq, layers[1], layers[2], layers[0], moment)
            + interpolate(xyz, tets, topo, e_dof, points))


def locate(xyz, tets, points, tol=1e-12):
    """Containing element and barycentric coordinates of each point: all
    lambda >= -tol, lowest element id on ties; -1 if outside the mesh."""
    vol, g, X = geometry(xyz, tets)
    pts = np.asarray(points, dtype=np.float64)
    lo = X.min(axis=1) - 1e-9
    hi = X.max(axis=1) + 1e-9
    elem = np.full(len(pts), -1, dtype=np.int64)
    lams = np.zeros((len(pts), 4))
    for r, p in enumerate(pts):
        cand = np.flatnonzero(np.all((p >= lo) & (p <= hi), axis=1))
        for e in cand:   # ascending ids
            lam = np.empty(4)
            lam[1:] = g[e, 1:] @ (p - X[e, 0])
            lam[0] = 1.0 - lam[1:].sum()
            if lam.min() >= -tol:
                elem[r] = e
                lams[r] = lam
                break
    return elem, lams


def interpolate(xyz, tets, topo: Topology, e_dof: np.ndarray, points) -> np.ndarray:
    """E(x) = sum_i N_i(x) e_i inside the containing element (Section 3, eq. 8);
    boundary edges carry zero. Returns complex128 [R][3]."""
    elem, lam = locate(xyz, tets, points)
    if np.any(elem < 0):
        raise ValueError("receiver outside the mesh")
    vol, g, X = geometry(xyz, np.asarray(tets)[elem])
    ell = edge_lengths(X)
    sign = topo.elem_sign[elem]
    N = basis_at(g, sign, ell, lam[:, None, :])[:, 0]                      # [R][6][3]
    dof = topo.dof_of_edge[topo.elem_edge[elem]]
    vals = np.where(dof >= 0, np.asarray(e_dof)[np.maximum(dof, 0)], 0.0)
    return np.einsum("rik,ri->rk", N, vals)


def receivers_total(xyz, tets, topo, e_dof, points, src_pos, src_dir, freq,
                    sigma_bg, moment=1.0) -> np.ndarray:
    """Total field E = E_p + E_s at the receivers (Section 2, eq. 4)."""
    return (dipole_field(points, src_pos, src_dir, freq, sigma_bg, moment)
            + interpolate(xyz, tets, topo, e_dof, points))


def curl_at(xyz, tets, topo: Topology, e_dof: np.ndarray, points) -> np.ndarray:
    """curl E = sum_i e_i curl N_i in the element containing each point, with
    curl N_i = 2 s_i l_i grad lambda_a x grad lambda_b (constant per element;
    Appendix B); boundary edges carry zero. Returns complex128 [R][3]."""
    elem, _ = locate(xyz, tets, points)
    if np.any(elem < 0):
        raise ValueError("receiver outside the mesh")
    vol, g, X = geometry(xyz, np.asarray(tets)[elem])
    ell = edge_lengths(X)
    sign = topo.elem_sign[elem]
    ea, eb = LOCAL_EDGES[:, 0], LOCAL_EDGES[:, 1]
    curl = 2.0 * (sign * ell)[:, :, None] * np.cross(g[:, ea], g[:, eb])     # [R][6][3]
    dof = topo.dof_of_edge[topo.elem_edge[elem]]
    vals = np.where(dof >= 0, np.asarray(e_dof)[np.maximum(dof, 0)], 0.0)
    return np.einsum("rik,ri->rk", curl, vals)


def receivers_total_h(xyz, tets, topo, e_dof, points, src_pos, src_dir, freq,
                      sigma_bg, moment=1.0) -> np.ndarray:
    """Total magnetic field H = H_p + curl E_s / (i omega mu0) at the receivers
    (Faraday's law, Section 2, eq. 1, e^{-i omega t})."""
    omega = 2.0 * np.pi * freq
    return (dipole_magnetic_field(points, src_pos, src_dir, freq, sigma_bg, moment)
            + curl_at(xyz, tets, topo, e_dof, points) / (1j * omega * MU0))


def receiver_error(E_test: np.ndarray, E_ref: np.ndarray) -> float:
    """max over receivers of |E_test - E_ref|_2 / |E_ref|_2 on complex
    3-vectors (a vector norm: single components may vanish by symmetry)."""
    num = np.sqrt(np.sum(np.abs(E_test - E_ref) ** 2, axis=-1))
    den = np.sqrt(np.sum(np.abs(E_ref) ** 2, axis=-1))
    return float(np.max(num / den))
