"""CPU checks of the COCG recurrences the GPU kernels use, in float64 on the
3,072-element block model (no GPU).

The fused step forms beta before r is updated, from the expansion
(r - alpha q)^T D^-1 (r - alpha q) = rho - 2 alpha q^T D^-1 r
+ alpha^2 q^T D^-1 q, and takes the exact r^T z of the new r for the next
alpha. In exact arithmetic this is the same recurrence as the plain Jacobi
COCG (rho' = r'^T z' after the update), so in float64 the two must give the
same iterates to rounding over the first iterations and converge alike."""
import numpy as np

from paper_1808_00186_amd import synth
from oracle import fem


def _system():
    m = synth.config1()
    s = fem.assemble(m.xyz, m.tets, m.sigma)
    d = m.sources[0]
    A = fem.system_matrix(s, d.freq).tocsr()
    b = fem.rhs(m.xyz, m.tets, m.sigma, m.sigma_bg, s.topo, d.pos, d.dir, d.freq, d.moment)
    return A, b


def _cocg(A, b, fused, iters):
    dinv = 1.0 / A.diagonal()
    x = np.zeros_like(b)
    r = b.copy()
    z = dinv * r
    p = z.copy()
    rho = r @ z
    xs, res = [], []
    for _ in range(iters):
        q = A @ p
        alpha = rho / (p @ q)
        if fused:
            beta = (rho - 2 * alpha * (q @ (dinv * r)) + alpha * alpha * (q @ (dinv * q))) / rho
            r = r - alpha * q
            z = dinv * r
            x = x + alpha * p
            p = z + beta * p
            rho = r @ z
        else:
            r = r - alpha * q
            z = dinv * r
            rho_new = r @ z
            beta = rho_new / rho
            rho = rho_new
            x = x + alpha * p
            p = z + beta * p
        xs.append(x.copy())
        res.append(np.linalg.norm(b - A @ x) / np.linalg.norm(b))
    return xs, res


def test_fused_beta_expansion_is_the_plain_recurrence():
    A, b = _system()
    xs_p, _ = _cocg(A, b, False, 40)
    xs_f, _ = _cocg(A, b, True, 40)
    for k in (0, 9, 19, 39):
        err = np.linalg.norm(xs_f[k] - xs_p[k]) / np.linalg.norm(xs_p[k])
        assert err < 1e-8, (k, err)


def test_fused_recurrence_converges_like_plain():
    A, b = _system()
    _, res_p = _cocg(A, b, False, 400)
    _, res_f = _cocg(A, b, True, 400)
    it_p = next(k for k, r in enumerate(res_p) if r <= 1e-8)
    it_f = next(k for k, r in enumerate(res_f) if r <= 1e-8)
    assert abs(it_f - it_p) <= max(2, it_p // 50), (it_p, it_f)
