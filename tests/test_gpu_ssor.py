"""The multicolour SSOR preconditioner (PETGEM_SSOR; the SOR family of the
paper's single-process solves, Section 5.3, Table 2) against the oracle's
definition (oracle/precond.py). Marked `gpu`.

* The colouring is a definition (greedy over the unknowns in the order of
  their global node pairs), so the library's colour of every edge must equal
  the oracle's, exactly.
* One application z = M^-1 r in complex64 against the oracle's complex128
  sweeps on the same r, element by element.
* Solves: COCG with SSOR in mixed precision on the small model with 1, 3 and
  9 sources (the few-column and the column-lane sweep kernels) and two
  relaxation factors, receivers within 1e-6 of the oracle at 1e-8, in fewer
  iterations than with Jacobi; and the 433,720-unknown marine model against
  its stored oracle fields at 1e-9.
* Every lane shape of Eisenstat's form (more than four columns): 8, 32 and
  64 lanes per row, the last with one, two and four columns per lane, exact
  fits and ragged tails, each column against the oracle.
* SQMR (the paper's solver with the SOR family): the same solves with the
  quasi-minimal-residual smoothing, in the explicit-product iteration (1 and
  3 sources) and in Eisenstat's form (9 and 33), against the oracle; it takes
  SSOR only, and the uneven batch refuses it.
"""
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fem, precond
from paper_1808_00186_amd import synth
from dofmap import lib_to_oracle

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def pg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1808_00186_amd import petgem
    petgem.lib()
    return petgem


def test_ssor_colouring_and_one_application_match_oracle(pg):
    import torch
    m = synth.config1()
    s = fem.assemble(m.xyz, m.tets, m.sigma)
    S = pg.System.from_model(m)
    perm = lib_to_oracle(S.dof_edges(), s.topo, len(m.xyz))
    print("[case] cfg1 SSOR colours and one application", flush=True)
    col_lib = S.ssor_colors()
    A = fem.system_matrix(s, 2.0)
    col_ref = precond.greedy_colors(A)
    col_o = np.empty_like(col_ref)
    col_o[perm] = col_lib
    assert np.array_equal(col_o, col_ref)
    rng = np.random.default_rng(11)
    r = (rng.standard_normal(S.n_dof) + 1j * rng.standard_normal(S.n_dof)).astype(np.complex64)
    for omega in (1.0, 1.25):
        z = S.ssor_apply(2.0, omega, torch.tensor(r, device="cuda")).cpu().numpy()
        r_o = np.empty(S.n_dof, np.complex128)
        r_o[perm] = r
        z_ref = precond.ssor_apply(A, col_ref, omega, r_o)[perm]
        err = np.abs(z - z_ref) / np.abs(z_ref).max()
        print(f"  omega {omega}: max element error {err.max():.2e} of max |z|", flush=True)
        assert err.max() <= 2e-5


@pytest.mark.parametrize("n_src", [1, 3, 9])
def test_cocg_ssor_matches_oracle_in_fewer_iterations(pg, n_src):
    m = synth.config1()
    xs = np.linspace(-300.0, 300.0, n_src)
    srcs = [synth.Dipole((float(x), 0.0, 300.0), f) for f in ((1.5,) if n_src < 9 else (0.5, 2.0, 3.0))
            for x in (xs if n_src < 9 else xs[:3])]
    s = fem.assemble(m.xyz, m.tets, m.sigma)
    ref = []
    lus = {}
    for d in srcs:
        if d.freq not in lus:
            lus[d.freq] = spla.splu(fem.system_matrix(s, d.freq).tocsc())
        b = fem.rhs(m.xyz, m.tets, m.sigma, m.sigma_bg, s.topo, d.pos, d.dir, d.freq, d.moment)
        ref.append(fem.receivers_total(m.xyz, m.tets, s.topo, lus[d.freq].solve(b), m.receivers, d.pos, d.dir,
                                       d.freq, m.sigma_bg, d.moment))
    S = pg.System.from_model(m)
    jac = pg.default_opts(method=pg.COCG, precision=pg.MIXED, rtol=1e-8, spmm_shape=0)
    _, st_j, _ = S.solve(srcs, jac)
    for omega in (1.0, 1.2):
        print(f"[case] cfg1 COCG SSOR omega {omega}, {len(srcs)} sources", flush=True)
        o = pg.default_opts(method=pg.COCG, precision=pg.MIXED, rtol=1e-8, precond=pg.SSOR, omega=omega)
        sol, st, rc = S.solve(srcs, o)
        assert rc == pg.OK and all(s_["rel_residual"] <= 1e-8 for s_ in st)
        E = sol.receivers(m.receivers).cpu().numpy()
        err = max(fem.receiver_error(E[k], ref[k]) for k in range(len(srcs)))
        it_s = max(s_["iters"] for s_ in st)
        it_j = max(s_["iters"] for s_ in st_j)
        print(f"  iters SSOR {it_s} Jacobi {it_j}, receiver error {err:.1e}", flush=True)
        assert err <= 1e-6
        assert it_s < it_j
    # the uneven batch and GMRES take Jacobi only
    with pytest.raises(pg.PetgemError):
        pg.solve_many([S], srcs[:1], pg.default_opts(method=pg.COCG, precision=pg.MIXED, precond=pg.SSOR))
    with pytest.raises(pg.PetgemError):
        S.solve(srcs[:1], pg.default_opts(precond=pg.SSOR))


def test_cocg_ssor_cfg2_matches_stored_oracle(pg):
    path = os.path.join(GOLDEN, "cfg2_receivers.npz")
    if not os.path.exists(path):
        pytest.skip("stored oracle fields missing")
    g = np.load(path)
    m = synth.config2()
    print("[case] cfg2 COCG SSOR", flush=True)
    S = pg.System.from_model(m)
    o = pg.default_opts(method=pg.COCG, precision=pg.MIXED, rtol=1e-9, precond=pg.SSOR)
    sol, st, rc = S.solve(m.sources, o)
    err = fem.receiver_error(sol.receivers(m.receivers).cpu().numpy()[0], g["E"])
    print(f"cfg2 COCG SSOR iters {st[0]['iters']} ir {st[0]['ir_steps']} res {st[0]['rel_residual']:.2e} "
          f"rx err {err:.2e} solve {st[0]['t_solve_ms']:.1f} ms", flush=True)
    assert rc == pg.OK and st[0]["rel_residual"] <= 1e-9
    assert err <= 1e-6


@pytest.fixture(scope="module")
def eis_pool():
    """200 sources on the small model (67 positions along x, each at 0.5, 1.5
    and 3 Hz, position-major) and the oracle's receiver fields of each."""
    m = synth.config1()
    xs = np.linspace(-400.0, 400.0, 67)
    srcs = [synth.Dipole((float(x), 0.0, 300.0), f) for x in xs for f in (0.5, 1.5, 3.0)][:200]
    s = fem.assemble(m.xyz, m.tets, m.sigma)
    lus, ref = {}, []
    for d in srcs:
        if d.freq not in lus:
            lus[d.freq] = spla.splu(fem.system_matrix(s, d.freq).tocsc())
        b = fem.rhs(m.xyz, m.tets, m.sigma, m.sigma_bg, s.topo, d.pos, d.dir, d.freq, d.moment)
        ref.append(fem.receivers_total(m.xyz, m.tets, s.topo, lus[d.freq].solve(b), m.receivers, d.pos, d.dir,
                                       d.freq, m.sigma_bg, d.moment))
    return m, srcs, ref


# columns -> Eisenstat sweep shape (lanes per row x columns per lane):
# 6 -> 8 x 1 (ragged), 32 -> 32 x 1 (exact), 64 -> 64 x 1 (exact),
# 100 -> 64 x 2 (ragged), 200 -> 64 x 4 (ragged)
@pytest.mark.parametrize("n_src", [6, 32, 64, 100, 200])
def test_eisenstat_lane_shapes_match_oracle(pg, eis_pool, n_src):
    m, pool, ref = eis_pool
    srcs = pool[:n_src]
    print(f"[case] cfg1 COCG SSOR (Eisenstat's form), {n_src} sources", flush=True)
    S = pg.System.from_model(m)
    o = pg.default_opts(method=pg.COCG, precision=pg.MIXED, rtol=1e-8, precond=pg.SSOR)
    sol, st, rc = S.solve(srcs, o)
    assert rc == pg.OK and all(s_["rel_residual"] <= 1e-8 for s_ in st)
    E = sol.receivers(m.receivers).cpu().numpy()
    errs = [fem.receiver_error(E[k], ref[k]) for k in range(n_src)]
    print(f"  iters max {max(s_['iters'] for s_ in st)}, receiver error max {max(errs):.1e}", flush=True)
    assert max(errs) <= 1e-6


@pytest.mark.parametrize("n_src", [1, 3, 9, 33])
def test_sqmr_ssor_matches_oracle(pg, eis_pool, n_src):
    m, pool, ref = eis_pool
    srcs = pool[:n_src]
    print(f"[case] cfg1 SQMR SSOR, {n_src} sources", flush=True)
    S = pg.System.from_model(m)
    o = pg.default_opts(method=pg.SQMR, precision=pg.MIXED, rtol=1e-8, precond=pg.SSOR)
    sol, st, rc = S.solve(srcs, o)
    assert rc == pg.OK and all(s_["rel_residual"] <= 1e-8 for s_ in st)
    E = sol.receivers(m.receivers).cpu().numpy()
    errs = [fem.receiver_error(E[k], ref[k]) for k in range(n_src)]
    oc = pg.default_opts(method=pg.COCG, precision=pg.MIXED, rtol=1e-8, precond=pg.SSOR)
    _, stc, _ = S.solve(srcs, oc)
    print(f"  iters SQMR {max(s_['iters'] for s_ in st)} COCG {max(s_['iters'] for s_ in stc)}, "
          f"receiver error max {max(errs):.1e}", flush=True)
    assert max(errs) <= 1e-6
    if n_src == 1:
        with pytest.raises(pg.PetgemError):   # SQMR takes SSOR
            S.solve(srcs, pg.default_opts(method=pg.SQMR, precision=pg.MIXED))
        with pytest.raises(pg.PetgemError):   # the uneven batch takes COCG with Jacobi
            pg.solve_many([S], srcs, pg.default_opts(method=pg.SQMR, precision=pg.MIXED, precond=pg.SSOR))
