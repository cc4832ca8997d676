"""Writes the stored oracle results used by the GPU parity tests at full size.

Calls only the CPU oracle (``oracle/``) and the seeded input generator; no
value comes from the GPU library. Run from the repository root:

    python tests/golden/make_golden.py cfg2

cfg2 -- the marine layered model (n = 40, 433,720 unknowns): receiver total and
secondary fields of its single source, solved by the oracle's Jacobi GMRES to
a true relative residual of 1e-12, plus the residual reached.
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import fem, solve  # noqa: E402
from paper_1808_00186_amd import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def cfg2():
    t0 = time.time()
    m = synth.config2()
    r = solve.forward(m, rtol=1e-12)
    np.savez_compressed(os.path.join(HERE, "cfg2_receivers.npz"), E=r["E"], Es=r["Es"],
                        residual=r["residual"], receivers=m.receivers,
                        n_dof=r["sys"].topo.n_dof, nnz=r["sys"].K.nnz)
    print(f"cfg2: {r['method']} residual {r['residual']:.3e} in {time.time() - t0:.1f} s")


if __name__ == "__main__":
    for name in sys.argv[1:] or ["cfg2"]:
        globals()[name]()
