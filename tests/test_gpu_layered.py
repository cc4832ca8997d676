"""The primary field over two half-spaces (sea over sediments) against the
oracle (oracle/layered.py and fem.rhs_layered). Marked `gpu`.

On a small marine model whose mesh follows the flat sea floor, the library's
right-hand side (dsigma at each quadrature point, the layered E_p summed by
Gauss-Legendre panels on the GPU) must equal the oracle's (own quadrature,
independent panels) within 1e-9 of its largest entry, and the total field at
the receivers after a solve within 1e-6, for x, y, z and tilted dipoles
through GMRES and the mixed COCG. A source at or below the interface and the
magnetic field over a layered background are refused.
"""
import numpy as np
import pytest

from oracle import fem, solve
from paper_1808_00186_amd import synth
from dofmap import lib_to_oracle

pytestmark = pytest.mark.gpu

TILT = tuple(np.array([0.3, -0.5, 0.81]) / np.linalg.norm([0.3, -0.5, 0.81]))


@pytest.fixture(scope="module")
def pg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1808_00186_amd import petgem
    petgem.lib()
    return petgem


@pytest.mark.parametrize("direction", [(1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0), TILT])
def test_layered_rhs_matches_oracle(pg, direction):
    m = synth.layered_marine(n=8, direction=direction)
    s = fem.assemble(m.xyz, m.tets, m.sigma)
    S = pg.System.from_model(m)
    perm = lib_to_oracle(S.dof_edges(), s.topo, len(m.xyz))
    src = m.sources[0]
    print(f"[case] layered rhs, dipole {direction}", flush=True)
    b = S.rhs(m.sources).cpu().numpy()[0]
    ref = fem.rhs_layered(m.xyz, m.tets, m.sigma, m.layers, s.topo, src.pos, src.dir, src.freq, src.moment)
    err = np.abs(b - ref[perm]).max() / np.abs(ref).max()
    print(f"  max error {err:.2e} of max |b|, nonzeros {np.count_nonzero(ref)}", flush=True)
    assert err <= 1e-9
    # the whole-space background of the same model is a different right-hand side
    S.set_background(None)
    b_ws = S.rhs(m.sources).cpu().numpy()[0]
    assert np.abs(b_ws - b).max() > 0.1 * np.abs(b).max()


@pytest.mark.parametrize("form", ["gmres", "cocg"])
def test_layered_solve_matches_oracle(pg, form):
    models = [synth.layered_marine(n=8, direction=d, freq=f) for d, f in
              (((1.0, 0.0, 0.0), 1.0), ((0.0, 0.0, 1.0), 0.4), (TILT, 1.7))]
    for m in models:
        ref = solve.forward(m)
        S = pg.System.from_model(m)
        o = (pg.default_opts(rtol=1e-9) if form == "gmres" else
             pg.default_opts(method=pg.COCG, precision=pg.MIXED, rtol=1e-9))
        print(f"[case] layered {form} dipole {m.sources[0].dir} f {m.sources[0].freq}", flush=True)
        sol, st, rc = S.solve(m.sources, o)
        assert rc == pg.OK and st[0]["rel_residual"] <= 1e-9
        E = sol.receivers(m.receivers).cpu().numpy()[0]
        err = fem.receiver_error(E, ref["E"])
        print(f"  iters {st[0]['iters']} receiver error {err:.2e} (oracle residual {ref['residual']:.1e})", flush=True)
        assert err <= 1e-6
        with pytest.raises(pg.PetgemError):
            sol.receivers_h(m.receivers)


def test_layered_refuses_a_source_below_the_interface(pg):
    m = synth.layered_marine(n=8, src=(0.0, 0.0, -40.0))
    S = pg.System.from_model(m)
    with pytest.raises(pg.PetgemError) as e:
        S.rhs(m.sources)
    assert e.value.code == pg.INVALID_ARG
