"""Maps the GPU library's DOF numbering onto the oracle's through the global
node pair of each interior edge (both number the same edges, in their own
orders)."""
import numpy as np


def lib_to_oracle(dof_edges: np.ndarray, topo, n_nodes: int) -> np.ndarray:
    """perm such that oracle_vector[perm] == library_vector."""
    okey = topo.edge_nodes[:, 0].astype(np.int64) * n_nodes + topo.edge_nodes[:, 1]
    lkey = dof_edges[:, 0].astype(np.int64) * n_nodes + dof_edges[:, 1]
    e = np.searchsorted(okey, lkey)
    assert np.all(okey[e] == lkey)
    perm = topo.dof_of_edge[e]
    assert np.all(perm >= 0)
    return perm


def csr_to_dense_coo(rp, col, val):
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    return rows, col, val
