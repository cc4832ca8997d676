"""GPU parity of the batched / mixed-precision forms against the CPU oracle.

The paper has no such forms (it solves one source at a time in double
precision), so their parity is pinned the same way as the plain path: the
receiver fields must match the oracle within 1e-6 (vector norm, max over
receivers) at the stated true relative residual, computed in double precision
on the GPU. Marked `gpu`.
"""
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fem, solve
from paper_1808_00186_amd import synth

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


def _oracle_fields(m, sources):
    """Oracle total fields [S][R][3]: one sparse LU per frequency."""
    s = fem.assemble(m.xyz, m.tets, m.sigma)
    out = []
    lus = {}
    for d in sources:
        if d.freq not in lus:
            lus[d.freq] = spla.splu(fem.system_matrix(s, d.freq).tocsc())
        b = fem.rhs(m.xyz, m.tets, m.sigma, m.sigma_bg, s.topo, d.pos, d.dir, d.freq, d.moment)
        x = lus[d.freq].solve(b)
        out.append(fem.receivers_total(m.xyz, m.tets, s.topo, x, m.receivers, d.pos, d.dir,
                                       d.freq, m.sigma_bg, d.moment))
    return np.array(out)


def _survey_sources(n_pos, freqs, z=300.0):
    xs = np.linspace(-400.0, 400.0, n_pos)
    return [synth.Dipole((float(x), 0.0, z), f) for f in freqs for x in xs]


@pytest.mark.parametrize("n_pos,freqs", [(1, (2.0,)), (5, (0.5, 2.0)), (11, (0.25, 1.0, 3.0))])
def test_cocg_mixed_multi_source_matches_oracle(pg, n_pos, freqs):
    m = synth.config1()
    srcs = _survey_sources(n_pos, freqs)
    print(f"[case] cfg1 COCG mixed C={len(srcs)}", flush=True)
    S = pg.System.from_model(m)
    o = pg.default_opts(method=pg.COCG, precision=pg.MIXED, rtol=1e-8)
    sol, st, rc = S.solve(srcs, o)
    assert rc == pg.OK
    E = sol.receivers(m.receivers).cpu().numpy()
    ref = _oracle_fields(m, srcs)
    errs = [fem.receiver_error(E[k], ref[k]) for k in range(len(srcs))]
    print(f"COCG C={len(srcs)} iters {[s['iters'] for s in st][:4]} ir {st[0]['ir_steps']} "
          f"max err {max(errs):.2e}", flush=True)
    assert all(s["rel_residual"] <= 1e-8 for s in st)
    assert max(errs) <= 1e-6


def test_cocg_matches_gmres_and_is_deterministic(pg):
    m = synth.config1()
    srcs = _survey_sources(3, (1.0,))
    S = pg.System.from_model(m)
    o = pg.default_opts(method=pg.COCG, precision=pg.MIXED, rtol=1e-10)
    s1, _, _ = S.solve(srcs, o)
    x1 = s1.x().cpu().numpy()
    s2, _, _ = S.solve(srcs, o)
    x2 = s2.x().cpu().numpy()
    assert np.array_equal(x1, x2)
    s3, _, _ = S.solve(srcs, pg.default_opts(method=pg.COCG, precision=pg.MIXED, rtol=1e-10, use_graph=0))
    assert np.array_equal(x1, s3.x().cpu().numpy())
    g, _, _ = S.solve(srcs, pg.default_opts(rtol=1e-10))
    xg = g.x().cpu().numpy()
    assert np.abs(x1 - xg).max() <= 1e-7 * np.abs(xg).max()


def test_cocg_initial_guess_and_fallback(pg):
    import torch
    m = synth.config1()
    srcs = _survey_sources(2, (2.0,))
    S = pg.System.from_model(m)
    o = pg.default_opts(method=pg.COCG, precision=pg.MIXED, rtol=1e-8)
    sol, st, _ = S.solve(srcs, o)
    x = sol.x()
    _, st2, _ = S.solve(srcs, o, x0=x)
    assert all(s["iters"] == 0 and s["used_fallback"] == 0 for s in st2)
    _, st3, _ = S.solve(srcs, o, x0=torch.full_like(x, float("nan")))
    assert all(s["used_fallback"] == 1 and s["rel_residual"] <= 1e-8 for s in st3)


def test_cocg_cfg2_single_source_matches_stored_oracle(pg):
    path = os.path.join(GOLDEN, "cfg2_receivers.npz")
    if not os.path.exists(path):
        pytest.skip("stored oracle fields missing")
    g = np.load(path)
    m = synth.config2()
    print("[case] cfg2 COCG mixed C=1", flush=True)
    S = pg.System.from_model(m)
    o = pg.default_opts(method=pg.COCG, precision=pg.MIXED, rtol=1e-9)
    sol, st, rc = S.solve(m.sources, o)
    err = fem.receiver_error(sol.receivers(m.receivers).cpu().numpy()[0], g["E"])
    print(f"cfg2 COCG mixed iters {st[0]['iters']} ir {st[0]['ir_steps']} res "
          f"{st[0]['rel_residual']:.2e} rx err {err:.2e} solve {st[0]['t_solve_ms']:.1f} ms", flush=True)
    assert rc == pg.OK and st[0]["rel_residual"] <= 1e-9
    # 1,695 tiles: the fused single-column step, whatever shape the tuner timed fastest
    assert st[0]["spmv_shape"] in (40104, 40108), st[0]["spmv_shape"]
    assert err <= 1e-6


# every complex64 SpMM shape the autotuner can pick, per column count, as the
# library lists them (petgem_spmm_candidates): 10000 kind + 100 a + b (kind 0
# CSR column lanes, 1 CSR nonzero lanes, 2 sliced ELLPACK, 3 pipelined sliced
# ELLPACK; one column of one mesh runs kind 3 as the fused step and reports
# kind 4), plus, for one column, the two fused steps forced with 4 and 8 slice
# columns in flight. 32 columns at one frequency is the block shape of the
# 6.9M-unknown survey; 33 columns over three frequencies leaves a ragged lane.
SHAPE_COLS = (1, 2, 3, 4, 32, 33)


def _shapes(pg, C):
    v = pg.spmm_candidates(C, C <= 4)
    if C == 1:
        v += [40104, 40108, 50104, 50108]
    return v


def _shape_sources(C):
    if C == 33:
        return _survey_sources(11, (0.25, 1.0, 3.0))
    if C == 32:
        return _survey_sources(32, (1.25,))
    return _survey_sources(C, (1.5,))


@pytest.mark.parametrize("C", SHAPE_COLS)
def test_every_spmm_shape_matches_oracle(pg, C):
    m = synth.config1()
    srcs = _shape_sources(C)
    ref = _oracle_fields(m, srcs)
    S = pg.System.from_model(m)
    shapes = _shapes(pg, C)
    assert shapes, C
    for shape in shapes:
        print(f"[case] cfg1 C={C} shape {shape}", flush=True)
        o = pg.default_opts(method=pg.COCG, precision=pg.MIXED, rtol=1e-8, spmm_shape=shape)
        sol, st, rc = S.solve(srcs, o)
        want = shape + 10000 if C == 1 and shape // 10000 == 3 else shape
        assert rc == pg.OK and all(s_["spmv_shape"] == want for s_ in st), (shape, st[0]["spmv_shape"])
        E = sol.receivers(m.receivers).cpu().numpy()
        err = max(fem.receiver_error(E[k], ref[k]) for k in range(len(srcs)))
        print(f"  shape {shape}: iters {st[0]['iters']} err {err:.1e}", flush=True)
        assert all(s_["rel_residual"] <= 1e-8 for s_ in st)
        assert err <= 1e-6
    with pytest.raises(pg.PetgemError):
        S.solve(srcs, pg.default_opts(method=pg.COCG, precision=pg.MIXED, spmm_shape=99999))
    if C > 1:   # the fused steps take one column only
        with pytest.raises(pg.PetgemError):
            S.solve(srcs, pg.default_opts(method=pg.COCG, precision=pg.MIXED, spmm_shape=40104))


def _small_marine(seed, n, f):
    xyz, tets = synth.kuhn_mesh(n, -5000.0, 5000.0, seed)
    rng = np.random.default_rng(seed)
    top = -float(rng.uniform(500, 2000))
    box = ((-1500, 1500), (-1500, 1500), (top - 300.0, top))
    sig = synth.marine_sigma(synth.centroids(xyz, tets), box, float(rng.uniform(0.005, 0.05)))
    rx = np.stack([np.linspace(-4000, 4000, 41), np.zeros(41), np.full(41, 10.0)], 1)
    return synth.Model(f"uneven-{seed}-n{n}", xyz, tets, sig, 3.3,
                       [synth.Dipole((float(rng.uniform(-1000, 1000)), 0.0, 50.0), f)], rx, n,
                       (-5000.0, 5000.0))


def test_solve_many_uneven_batch_matches_oracle(pg):
    models = [_small_marine(100 + k, n, f) for k, (n, f) in
              enumerate([(6, 0.3), (9, 1.7), (4, 0.9), (12, 0.5), (7, 1.1)])]
    print(f"[case] uneven batch sizes {[len(mm.tets) for mm in models]}", flush=True)
    systems = [pg.System.from_model(mm) for mm in models]
    o = pg.default_opts(method=pg.COCG, precision=pg.MIXED, rtol=1e-9)
    sols, st, rc = pg.solve_many(systems, [mm.sources[0] for mm in models], o)
    assert rc == pg.OK
    # one column per mesh takes the fused step with a reduction block per mesh
    assert all(s_["spmv_shape"] in (50104, 50108) for s_ in st), [s_["spmv_shape"] for s_ in st]
    for k, mm in enumerate(models):
        E = sols[k].receivers(mm.receivers).cpu().numpy()[0]
        ref = solve.forward(mm)["E"]
        err = fem.receiver_error(E, ref)
        print(f"  model {k} n={mm.n} iters {st[k]['iters']} res {st[k]['rel_residual']:.1e} err {err:.1e}",
              flush=True)
        assert st[k]["rel_residual"] <= 1e-9
        assert err <= 1e-6
    # the same batch again reuses the captured graph and gives identical results
    sols2, _, _ = pg.solve_many(systems, [mm.sources[0] for mm in models], o)
    for a, b in zip(sols, sols2):
        assert np.array_equal(a.x().cpu().numpy(), b.x().cpu().numpy())
    # initial guesses per system: the solution itself (no iterations), none,
    # and a non-finite one (replaced by zero for that system alone)
    import torch
    xs = [s_.x()[0] for s_ in sols]
    x0 = [xs[0], None, torch.full_like(xs[2], float("nan")), xs[3] * 1e3, xs[4]]
    sols3, st3, rc3 = pg.solve_many(systems, [mm.sources[0] for mm in models], o, x0=x0)
    assert rc3 == pg.OK
    print(f"  x0 batch: iters {[s_['iters'] for s_ in st3]} fallback {[s_['used_fallback'] for s_ in st3]}",
          flush=True)
    assert st3[0]["iters"] == 0 and st3[4]["iters"] == 0 and st3[3]["iters"] == 0
    assert [s_["used_fallback"] for s_ in st3] == [0, 0, 1, 0, 0]
    assert st3[1]["iters"] > 0 and st3[2]["iters"] > 0
    for k, mm in enumerate(models):
        E = sols3[k].receivers(mm.receivers).cpu().numpy()[0]
        assert st3[k]["rel_residual"] <= 1e-9
        assert fem.receiver_error(E, solve.forward(mm)["E"]) <= 1e-6


def test_uneven_batch_of_smallest_cfg4_models_matches_oracle(pg):
    """The four smallest models of the 48-model uneven batch (coarse meshes,
    h up to 833 m) and the smallest 1.8 Hz one, against the oracle at the true
    residual the batch is run at, 1e-12 (1e-10 still leaves up to 1e-5 at the
    far receivers of the high-frequency models)."""
    models = synth.config4()
    small = sorted(models, key=lambda m: len(m.tets))[:4]
    small.append(min((m for m in models if m.sources[0].freq > 1.75), key=lambda m: len(m.tets)))
    print(f"[case] cfg4 small models {[len(m.tets) for m in small]}", flush=True)
    systems = [pg.System.from_model(m) for m in small]
    o = pg.default_opts(method=pg.COCG, precision=pg.MIXED, rtol=1e-12)
    sols, st, rc = pg.solve_many(systems, [m.sources[0] for m in small], o)
    assert rc == pg.OK
    assert all(s_["spmv_shape"] in (50104, 50108) for s_ in st), [s_["spmv_shape"] for s_ in st]
    for k, m in enumerate(small):
        E = sols[k].receivers(m.receivers).cpu().numpy()[0]
        err = fem.receiver_error(E, solve.forward(m)["E"])
        print(f"  {m.name} tets {len(m.tets)} f {m.sources[0].freq:.2f} iters {st[k]['iters']} "
              f"res {st[k]['rel_residual']:.1e} err {err:.1e}", flush=True)
        assert st[k]["rel_residual"] <= 1e-12 and err <= 1e-6


@pytest.mark.parametrize("seeds", [(4018, 4047)])
def test_uneven_batch_of_largest_and_hardest_cfg4_models_matches_stored_oracle(pg, seeds):
    """The largest model of the 48-model uneven batch (seed 4018, 1,361,886
    elements) and the slowest to converge (seed 4047, 1,296,000 elements at
    0.61 Hz), solved together as one uneven batch at the batch's residual of
    1e-12, against the oracle's receiver fields (Jacobi GMRES to 1e-12,
    tests/golden/cfg4_<seed>.npz, written by the oracle only)."""
    paths = [os.path.join(GOLDEN, f"cfg4_{sd}.npz") for sd in seeds]
    if not all(os.path.exists(p) for p in paths):
        pytest.skip("stored oracle fields missing")
    models = [synth.config4_model(sd) for sd in seeds]
    print(f"[case] cfg4 models {seeds}: {[len(m.tets) for m in models]} elements", flush=True)
    systems = [pg.System.from_model(m) for m in models]
    o = pg.default_opts(method=pg.COCG, precision=pg.MIXED, rtol=1e-12)
    sols, st, rc = pg.solve_many(systems, [m.sources[0] for m in models], o)
    assert rc == pg.OK
    for k, (m, p) in enumerate(zip(models, paths)):
        g = np.load(p)
        E = sols[k].receivers(m.receivers).cpu().numpy()[0]
        err = fem.receiver_error(E, g["E"])
        print(f"  {m.name}: iters {st[k]['iters']} res {st[k]['rel_residual']:.1e} (oracle {float(g['residual']):.1e}) "
              f"err {err:.1e}", flush=True)
        assert st[k]["rel_residual"] <= 1e-12 and err <= 1e-6


def test_phase_separation_probe(pg):
    """The measurement behind the uneven batch's graph-replayed kernels: both
    probes run and report a positive time per round; the persistent form
    fills the GPU with resident blocks."""
    us0, b0 = pg.sync_probe(200, 0)
    us1, b1 = pg.sync_probe(200, 1)
    print(f"graph kernel boundary {us0:.2f} us, grid barrier {us1:.2f} us ({b1} blocks)", flush=True)
    assert us0 > 0 and us1 > 0 and b1 >= 256
    with pytest.raises(pg.PetgemError):
        pg.sync_probe(0, 0)
