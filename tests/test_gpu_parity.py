"""GPU parity of the HIP path against the CPU oracle, stage by stage, through
the C ABI (ctypes binding). Marked `gpu`: needs an MI355X and the built
library.

Tolerances (double precision everywhere on this path):
  assembly K, M_sigma   max|gpu - oracle| <= 1e-12 max|oracle|
  right-hand side       max|gpu - oracle| <= 1e-12 max|oracle|
  A x (SpMV)            max|gpu - oracle| <= 1e-13 max|oracle|
  receivers             max_r |E_gpu - E_ora|_2 / |E_ora|_2 <= 1e-6 at a true
                        relative residual <= 1e-8 (the oracle solves directly
                        or to 1e-12)
The assembled values and the solution must also be bitwise reproducible, and
K, M_sigma bitwise symmetric.
"""
import os

import numpy as np
import pytest

from dofmap import lib_to_oracle
from oracle import fem, solve
from paper_1808_00186_amd import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def pg():
    from paper_1808_00186_amd import petgem
    petgem.lib()
    return petgem


def _case(model):
    print(f"[case] {model.name} T={len(model.tets)}", flush=True)


def _oracle(model):
    s = fem.assemble(model.xyz, model.tets, model.sigma)
    return s


def _dense_sym(rp, col, val, n):
    A = np.zeros((n, n))
    rows = np.repeat(np.arange(n), np.diff(rp))
    A[rows, col] = val
    return A


@pytest.mark.parametrize("which", ["cfg1", "tiny3", "ragged5"])
def test_assembly_matches_oracle_and_is_symmetric(torch_cuda, pg, which):
    if which == "cfg1":
        m = synth.config1()
    else:
        n = 3 if which == "tiny3" else 5
        xyz, tets = synth.kuhn_mesh(n, -700.0, 900.0, 40 + n)
        sig = np.random.default_rng(n).uniform(0.01, 3.3, len(tets))
        m = synth.Model(which, xyz, tets, sig, 1.0, [synth.Dipole((10.0, 20.0, 30.0), 1.0)],
                        np.zeros((1, 3)), n, (-700.0, 900.0))
    _case(m)
    S = pg.System.from_model(m)
    rp, col, K, Ms = S.csr()
    ref = _oracle(m)
    perm = lib_to_oracle(S.dof_edges(), ref.topo, len(m.xyz))
    rows = np.repeat(np.arange(S.n_dof), np.diff(rp))
    Ko = np.asarray(ref.K[perm[rows], perm[col]]).ravel()
    Mo = np.asarray(ref.Ms[perm[rows], perm[col]]).ravel()
    assert np.abs(K - Ko).max() <= 1e-12 * np.abs(Ko).max()
    assert np.abs(Ms - Mo).max() <= 1e-12 * np.abs(Mo).max()
    # bitwise symmetry of the deterministic gather
    key = rows.astype(np.int64) * S.n_dof + col
    tkey = col.astype(np.int64) * S.n_dof + rows
    idx = np.searchsorted(key, tkey)
    assert np.array_equal(K[idx], K) and np.array_equal(Ms[idx], Ms)


def test_assembly_bitwise_reproducible_and_reassemble(torch_cuda, pg):
    torch = torch_cuda
    m = synth.config1()
    _case(m)
    S = pg.System.from_model(m)
    _, _, K1, M1 = S.csr()
    S.reassemble(torch.tensor(m.sigma, device="cuda"), m.sigma_bg)
    _, _, K2, M2 = S.csr()
    assert np.array_equal(K1, K2) and np.array_equal(M1, M2)
    # new conductivities through the device-only path
    sig2 = m.sigma * 2.0
    S.reassemble(torch.tensor(sig2, device="cuda"), m.sigma_bg)
    rp, col, K3, M3 = S.csr()
    assert np.array_equal(K3, K1)
    ref = fem.assemble(m.xyz, m.tets, sig2)
    perm = lib_to_oracle(S.dof_edges(), ref.topo, len(m.xyz))
    rows = np.repeat(np.arange(S.n_dof), np.diff(rp))
    Mo = np.asarray(ref.Ms[perm[rows], perm[col]]).ravel()
    assert np.abs(M3 - Mo).max() <= 1e-12 * np.abs(Mo).max()


@pytest.mark.parametrize("cfg", ["cfg1", "cfg5-10007"])
def test_rhs_matches_oracle(torch_cuda, pg, cfg):
    m = synth.config1() if cfg == "cfg1" else synth.config5_sample(10007)
    _case(m)
    S = pg.System.from_model(m)
    srcs = list(m.sources) + [synth.Dipole((55.0, -40.0, 330.0), 0.7, (0.0, 0.6, 0.8), 2.5)]
    b = S.rhs(srcs).cpu().numpy()
    ref = _oracle(m)
    perm = lib_to_oracle(S.dof_edges(), ref.topo, len(m.xyz))
    for k, s in enumerate(srcs):
        bo = fem.rhs(m.xyz, m.tets, m.sigma, m.sigma_bg, ref.topo, s.pos, s.dir, s.freq, s.moment)
        assert np.abs(bo).max() > 0
        assert np.abs(b[k] - bo[perm]).max() <= 1e-12 * np.abs(bo).max()


def test_spmv_matches_oracle(torch_cuda, pg):
    torch = torch_cuda
    m = synth.config1()
    _case(m)
    S = pg.System.from_model(m)
    ref = _oracle(m)
    perm = lib_to_oracle(S.dof_edges(), ref.topo, len(m.xyz))
    rng = np.random.default_rng(5)
    x = rng.normal(size=S.n_dof) + 1j * rng.normal(size=S.n_dof)
    for f in (0.25, 2.0):
        y = S.spmv(f, torch.tensor(x, device="cuda")).cpu().numpy()
        A = fem.system_matrix(ref, f)
        xo = np.empty_like(x)
        xo[perm] = x
        yo = (A @ xo)[perm]
        assert np.abs(y - yo).max() <= 1e-13 * np.abs(yo).max()


def _solve_and_compare(pg, m, opts=None, tol=1e-6):
    S = pg.System.from_model(m)
    sol, stats, rc = S.solve(m.sources, opts)
    E = sol.receivers(m.receivers).cpu().numpy()
    x = sol.x().cpu().numpy()
    ref = solve.forward(m)
    err = fem.receiver_error(E[0], ref["E"])
    # true residual of the GPU solution with the oracle's own A and b
    perm = lib_to_oracle(S.dof_edges(), ref["sys"].topo, len(m.xyz))
    xo = np.empty_like(x[0])
    xo[perm] = x[0]
    res = np.linalg.norm(ref["b"] - ref["A"] @ xo) / np.linalg.norm(ref["b"])
    return S, sol, stats, err, res, ref, E


def test_cfg1_receivers_match_oracle(torch_cuda, pg):
    m = synth.config1()
    _case(m)
    S, sol, stats, err, res, ref, E = _solve_and_compare(pg, m)
    print(f"cfg1 gmres iters {stats[0]['iters']} res {stats[0]['rel_residual']:.2e} "
          f"oracle-res {res:.2e} rx err {err:.2e}", flush=True)
    assert stats[0]["rel_residual"] <= 1e-8 and res <= 1.5e-8
    assert err <= 1e-6


def test_cfg1_solution_bitwise_reproducible(torch_cuda, pg):
    m = synth.config1()
    _case(m)
    S = pg.System.from_model(m)
    sol1, _, _ = S.solve(m.sources)
    x1 = sol1.x().cpu().numpy()
    sol2, _, _ = S.solve(m.sources, solution=sol1)
    x2 = sol2.x().cpu().numpy()
    sol3, _, _ = S.solve(m.sources, pg.default_opts(use_graph=0))
    x3 = sol3.x().cpu().numpy()
    assert np.array_equal(x1, x2) and np.array_equal(x1, x3)


@pytest.mark.parametrize("shape", [0, 20104, 30104])
def test_mixed_solution_bitwise_reproducible(torch_cuda, pg, shape):
    """Mixed COCG: graph replay with the overlapped host checks and the
    synchronous loop without graphs run the same iterations (convergence is
    decided on the device), so the solutions agree bitwise. Shape 0 is the
    tuned one, 20104 the two-vector-kernel step, 30104 the fused step."""
    m = synth.config1()
    _case(m)
    S = pg.System.from_model(m)
    kw = dict(method=pg.COCG, precision=pg.MIXED, spmm_shape=shape)
    sol1, st1, _ = S.solve(m.sources, pg.default_opts(**kw))
    x1 = sol1.x().cpu().numpy()
    sol2, st2, _ = S.solve(m.sources, pg.default_opts(**kw), solution=sol1)
    x2 = sol2.x().cpu().numpy()
    sol3, st3, _ = S.solve(m.sources, pg.default_opts(use_graph=0, **kw))
    x3 = sol3.x().cpu().numpy()
    assert st1[0]["iters"] == st2[0]["iters"] == st3[0]["iters"]
    assert np.array_equal(x1, x2) and np.array_equal(x1, x3)
    # a chosen shape is honoured; tuned, one column always takes the fused step
    assert st1[0]["spmv_shape"] == {0: 40104, 30104: 40104}.get(shape, shape)
    assert st1[0]["rel_residual"] <= 1e-8


def test_initial_guess_and_fallback(torch_cuda, pg):
    torch = torch_cuda
    m = synth.config1()
    _case(m)
    S = pg.System.from_model(m)
    sol, st, _ = S.solve(m.sources)
    x = sol.x()
    # the converged solution as a guess: no iteration needed
    _, st2, _ = S.solve(m.sources, x0=x)
    assert st2[0]["iters"] == 0 and st2[0]["used_fallback"] == 0
    # a non-finite guess falls back to zero and still converges
    sol3, st3, _ = S.solve(m.sources, x0=torch.full_like(x, float("nan")))
    assert st3[0]["used_fallback"] == 1 and st3[0]["rel_residual"] <= 1e-8
    assert st3[0]["iters"] == st[0]["iters"]
    # a badly scaled guess is rescaled by the alpha minimising |b - alpha A x0|
    _, st4, _ = S.solve(m.sources, x0=(x * 1e6).contiguous())
    assert st4[0]["used_fallback"] == 0 and st4[0]["iters"] == 0


def test_not_converged_and_zero_rhs(torch_cuda, pg):
    m = synth.config1()
    _case(m)
    S = pg.System.from_model(m)
    sol, st, rc = S.solve(m.sources, pg.default_opts(max_iter=2, restart=2), allow_not_converged=True)
    assert rc == pg.NOT_CONVERGED and st[0]["status"] == pg.NOT_CONVERGED
    assert st[0]["rel_residual"] > 1e-8
    # no anomaly: b = 0, x = 0
    m0 = synth.Model("uniform", m.xyz, m.tets, np.ones(len(m.tets)), 1.0, m.sources, m.receivers)
    S0 = pg.System.from_model(m0)
    sol0, st0, rc0 = S0.solve(m0.sources)
    assert rc0 == pg.OK and np.all(sol0.x().cpu().numpy() == 0)


def test_receiver_outside_and_singular_source(torch_cuda, pg):
    m = synth.config1()
    _case(m)
    S = pg.System.from_model(m)
    sol, _, _ = S.solve(m.sources)
    with pytest.raises(pg.PetgemError) as e:
        sol.receivers(np.array([[0.0, 0.0, 5000.0]]))
    assert e.value.code == pg.RECEIVER_OUTSIDE
    # a source on a quadrature point of an element inside the anomaly
    ref = _oracle(m)
    t = int(np.flatnonzero(m.sigma != m.sigma_bg)[0])
    xq = fem.QUAD4[0] @ m.xyz[m.tets[t]]
    with pytest.raises(pg.PetgemError) as e:
        S.solve([synth.Dipole(tuple(xq), 1.0)])
    assert e.value.code == pg.SOURCE_SINGULAR


def test_cfg2_receivers_match_stored_oracle(torch_cuda, pg):
    """Full-size marine model (433,720 unknowns) against the oracle's stored
    receiver fields (written by tests/golden/make_golden.py, oracle only).

    At a true relative residual of 1e-8 the receiver error on this model is
    about 2e-6 (the far receivers see a small total field), so this workload
    is solved to 1e-9, which gives about 2e-7; the 1e-8 result is printed."""
    path = os.path.join(GOLDEN, "cfg2_receivers.npz")
    if not os.path.exists(path):
        pytest.skip("stored oracle fields missing")
    g = np.load(path)
    m = synth.config2()
    _case(m)
    S = pg.System.from_model(m)
    assert S.n_dof == int(g["n_dof"]) and S.nnz == int(g["nnz"])
    sol8, st8, _ = S.solve(m.sources, pg.default_opts(rtol=1e-8))
    err8 = fem.receiver_error(sol8.receivers(m.receivers).cpu().numpy()[0], g["E"])
    sol, st, rc = S.solve(m.sources, pg.default_opts(rtol=1e-9))
    E, Es = sol.receivers(m.receivers, secondary=True)
    err = fem.receiver_error(E.cpu().numpy()[0], g["E"])
    print(f"cfg2 gmres rtol 1e-8: iters {st8[0]['iters']} rx err {err8:.2e}; rtol 1e-9: iters "
          f"{st[0]['iters']} res {st[0]['rel_residual']:.2e} rx err {err:.2e} "
          f"solve {st[0]['t_solve_ms']:.1f} ms", flush=True)
    assert st[0]["rel_residual"] <= 1e-9
    assert err <= 1e-6
    # the true residual of the GPU solution with the oracle's own A and b
    ref = fem.assemble(m.xyz, m.tets, m.sigma)
    src = m.sources[0]
    A = fem.system_matrix(ref, src.freq)
    b = fem.rhs(m.xyz, m.tets, m.sigma, m.sigma_bg, ref.topo, src.pos, src.dir, src.freq)
    perm = lib_to_oracle(S.dof_edges(), ref.topo, len(m.xyz))
    xo = np.empty(S.n_dof, dtype=complex)
    xo[perm] = sol.x().cpu().numpy()[0]
    res = np.linalg.norm(b - A @ xo) / np.linalg.norm(b)
    assert res <= 1.5e-9, res
