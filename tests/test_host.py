"""CPU tests of the library's host side: the C ABI loads and exports every
declared entry point, and the host preprocessing (edge numbering, boundary
elimination, CSR pattern, point location) matches the oracle's own,
independently computed topology exactly. No GPU call is made here."""
import os
import re

import numpy as np
import pytest

from paper_1808_00186_amd import petgem, synth
from oracle import fem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "petgem.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(petgem_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = petgem.lib()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert set(names) >= set(petgem._SIGS), set(petgem._SIGS) - set(names)


def test_binding_constants_match_header():
    txt = open(os.path.join(ROOT, "include", "petgem.h")).read()
    defs = {k: int(v) for k, v in re.findall(r"#define\s+PETGEM_([A-Z0-9_]+)\s+(-?\d+)", txt)}
    for name in ("GMRES", "COCG", "BCOCG", "SQMR", "JACOBI", "SSOR", "FP64", "MIXED", "OK"):
        assert getattr(petgem, name) == defs[name], name


def _oracle_pattern(xyz, tets):
    s = fem.assemble(xyz, tets, np.ones(len(tets)))
    return s.topo, s.K.tocsr()


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (3, 2), (5, 3), (8, 1)])
def test_pattern_matches_oracle(n, seed):
    xyz, tets = synth.kuhn_mesh(n, -1000.0, 1000.0, seed)
    de, rp, col = petgem.mesh_pattern(xyz, tets)
    topo, K = _oracle_pattern(xyz, tets)
    assert len(de) == topo.n_dof
    assert np.all(de[:, 0] < de[:, 1])
    # map library DOFs to oracle DOFs through the global node pairs
    N = len(xyz)
    okey = topo.edge_nodes[:, 0] * N + topo.edge_nodes[:, 1]
    lkey = de[:, 0].astype(np.int64) * N + de[:, 1]
    eidx = np.searchsorted(okey, lkey)
    assert np.all(okey[eidx] == lkey)
    odof = topo.dof_of_edge[eidx]
    assert np.all(odof >= 0) and len(np.unique(odof)) == topo.n_dof
    rows = np.repeat(np.arange(len(de)), np.diff(rp))
    assert np.all(np.diff(col)[np.diff(rows) == 0] > 0)       # sorted, unique per row
    lib_pairs = set(zip(odof[rows].tolist(), odof[col].tolist()))
    Kc = K.tocoo()
    assert lib_pairs == set(zip(Kc.row.tolist(), Kc.col.tolist()))


def test_config_sizes_exact():
    for cfg, (ndof, nnz) in ((synth.config1(), (3032, 43688)),):
        de, rp, col = petgem.mesh_pattern(cfg.xyz, cfg.tets)
        assert (len(de), len(col)) == (ndof, nnz)


@pytest.mark.slow
def test_cfg2_sizes_exact():
    m = synth.config2()
    de, rp, col = petgem.mesh_pattern(m.xyz, m.tets)
    assert (len(de), len(col)) == (433720, 6950152)


def test_locate_matches_oracle():
    m = synth.config1()
    rng = np.random.default_rng(0)
    pts = np.concatenate([m.receivers, rng.uniform(-999, 999, (30, 3))])
    got = petgem.locate(m.xyz, m.tets, pts)
    ref, _ = fem.locate(m.xyz, m.tets, pts)
    assert np.array_equal(got, ref)


def test_locate_tie_break_and_outside():
    xyz, tets = synth.kuhn_mesh(1, 0.0, 1.0, None)
    got = petgem.locate(xyz, tets, np.array([[0.3, 0.3, 0.3], [2.0, 0.5, 0.5], [0.0, 0.0, 0.0]]))
    ref, _ = fem.locate(xyz, tets, np.array([[0.3, 0.3, 0.3], [2.0, 0.5, 0.5], [0.0, 0.0, 0.0]]))
    assert got.tolist() == ref.tolist() == [0, -1, 0]


def test_error_paths():
    xyz, tets = synth.kuhn_mesh(2, 0.0, 1.0, 3)
    bad = tets.copy()
    bad[5, 3] = len(xyz) + 10
    with pytest.raises(petgem.PetgemError) as e:
        petgem.mesh_pattern(xyz, bad)
    assert e.value.code == petgem.INVALID_ARG
    flat = xyz.copy()
    flat[tets[0]] = flat[tets[0, 0]] + np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]]) * 0.1
    with pytest.raises(petgem.PetgemError) as e:
        petgem.mesh_pattern(flat, tets)
    assert e.value.code == petgem.DEGENERATE_ELEMENT
    # a third element on an existing face
    extra = np.concatenate([tets, tets[:1]])
    with pytest.raises(petgem.PetgemError) as e:
        petgem.mesh_pattern(xyz, extra)
    assert e.value.code == petgem.MESH_TOPOLOGY


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus above 1 exits with a message before
    touching a device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_bench_names_and_prices_the_fused_product():
    """The roofline entry of bench.py: shape 40104 (the fused step's product)
    is named after its kernel, charged 16 B per row more than the plain
    sliced-ELLPACK product (r and D^-1), and has a measured traffic figure."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    n, nnz = 433720, 6950152
    assert bench.spmm_bytes_fp32(n, nnz, 1, 40104) == 12 * nnz + 36 * n == 99015744
    assert bench.spmm_bytes_fp32(n, nnz, 1, 30104) == 12 * nnz + 20 * n
    name = bench.kernel_name("mixed", 40104)
    assert name.startswith("k_spmm_spb<4, 4>")
    assert name in bench.MEASURED_TRAFFIC
    assert bench.kernel_name("mixed", 30104).startswith("k_spmm_sp<1, 4>")
    assert bench.kernel_name("plain", 8).startswith("k_spmv<8, false>")


def test_spmm_candidates_listed_by_the_library():
    """The autotuner's shape lists (host only): sliced ELLPACK only with the
    sliced copy and up to four columns, column lanes (also with the row's
    entries spread over the lanes, kind 6, up to 64 columns) from four columns
    on, every list non-empty, and a column lane layout always covers the
    block."""
    for C in (1, 2, 3, 4, 5, 8, 16, 32, 33, 96, 300):
        for sliced in (False, True):
            v = petgem.spmm_candidates(C, sliced)
            assert v, (C, sliced)
            for code in v:
                kind, a, b = code // 10000, code // 100 % 100, code % 100
                assert kind in (0, 1, 2, 3, 6)
                if kind in (2, 3):
                    assert sliced and C <= 4
                if kind == 0:
                    assert C >= 4 and (a * b >= C or (a, b) == (64, 4))
                if kind == 6:
                    assert 4 <= C <= 64 and a * b >= C
                if kind == 1:
                    assert C <= 4
    with pytest.raises(petgem.PetgemError):
        petgem.spmm_candidates(0, False)


def test_default_options():
    """petgem_default_opts fills every field as its header states."""
    o = petgem.default_opts()
    assert (o.method, o.precision, o.restart, o.max_iter) == (petgem.GMRES, petgem.FP64, 30, 20000)
    assert (o.rtol, o.inner_rtol, o.use_graph, o.profile, o.verbose, o.spmm_shape) == (1e-8, 3e-5, 1, 0, 0, 0)
    assert (o.precond, o.omega) == (petgem.JACOBI, 1.0)
