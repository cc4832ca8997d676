"""Seeded synthetic marine-CSEM workloads: jittered Kuhn tetrahedral meshes,
per-element conductivity models, dipole sources and receiver lines.

This module only *builds inputs*. It holds none of the method's arithmetic
(no basis functions, no element matrices, no primary field, no solver), so the
CPU oracle and the GPU library can both take their inputs from it without
sharing any part of the computation.

The paper meshes its models with Gmsh (Section 4, parameters file) and adapts
the spacing to the skin depth (Section 5.3, eqs. 12-17). Those meshes are not
available, so the workloads here are uniform hexahedral grids split into six
tetrahedra each, with every interior vertex jittered, which keeps the meshes
unstructured in the sense that matters for the kernels (irregular element
shapes, edge valences from 4 to 14, irregular CSR rows).

Recipe (all sizes in metres, conductivities in S/m, frequencies in Hz):

* Nodes of an n x n x n grid over ``[lo, hi]^3`` are numbered i-major, then j,
  then k. One ``numpy.random.default_rng(seed).uniform(-0.15h, 0.15h, (N, 3))``
  draw jitters every coordinate; the component normal to a boundary face the
  node lies on is zeroed so that the box stays a box.
* Each hexahedron (i-major order) is split into six tetrahedra along its
  (0,0,0)->(1,1,1) diagonal, one per axis permutation in the order
  (x,y,z), (x,z,y), (y,x,z), (y,z,x), (z,x,y), (z,y,x); the split is conforming.
* The conductivity of an element is that of the region containing its
  centroid: boxes are closed on every axis, a reservoir box overrides the
  layers, sea water is centroid z > 0 and sediments z <= 0.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

# Axis permutations of the six Kuhn tetrahedra of one hexahedron.
_KUHN_PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))


@dataclass
class Dipole:
    """A point electric dipole: position (m), unit direction, frequency (Hz)
    and moment I*dS (A*m)."""
    pos: Tuple[float, float, float]
    freq: float
    dir: Tuple[float, float, float] = (1.0, 0.0, 0.0)
    moment: float = 1.0


@dataclass
class Model:
    """One forward-modelling problem: mesh, conductivities, sources, receivers."""
    name: str
    xyz: np.ndarray            # float64 [N][3]
    tets: np.ndarray           # int32 [T][4]
    sigma: np.ndarray          # float64 [T] total conductivity per element
    sigma_bg: float            # background conductivity of the primary field
    sources: List[Dipole]
    receivers: np.ndarray      # float64 [R][3]
    n: int = 0                 # hexahedra per side
    box: Tuple[float, float] = (0.0, 0.0)
    meta: dict = field(default_factory=dict)
    # background of the primary field: None = the whole space sigma_bg;
    # (z0, sigma_above, sigma_below) = two half-spaces meeting at z = z0
    layers: Optional[Tuple[float, float, float]] = None

    @property
    def h(self) -> float:
        return (self.box[1] - self.box[0]) / self.n


def kuhn_mesh(n: int, lo: float, hi: float, seed: Optional[int],
              jitter: float = 0.15, flat_z: Tuple[float, ...] = ()) -> Tuple[np.ndarray, np.ndarray]:
    """Jittered Kuhn mesh of the cube [lo, hi]^3 with n hexahedra per side.

    Returns (xyz float64 [(n+1)^3][3], tets int32 [6 n^3][4]).
    ``seed=None`` gives the unjittered grid. Nodes of the grid planes
    z = c for c in ``flat_z`` keep their z (jittered in x and y only), so a
    layer interface there is matched by element faces."""
    if n < 1:
        raise ValueError("n must be >= 1")
    h = (hi - lo) / n
    m = n + 1
    ijk = np.stack(np.meshgrid(np.arange(m), np.arange(m), np.arange(m),
                               indexing="ij"), axis=-1).reshape(-1, 3)
    xyz = lo + h * ijk.astype(np.float64)
    if seed is not None and jitter != 0.0:
        rng = np.random.default_rng(seed)
        jit = rng.uniform(-jitter * h, jitter * h, size=xyz.shape)
        jit[(ijk == 0) | (ijk == n)] = 0.0
        for c in flat_z:
            jit[np.isclose(xyz[:, 2], c), 2] = 0.0
        xyz = xyz + jit

    def nid(i, j, k):
        return (i * m + j) * m + k

    hi_ = np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n),
                               indexing="ij"), axis=-1).reshape(-1, 3)
    tets = np.empty((hi_.shape[0], 6, 4), dtype=np.int64)
    for t, perm in enumerate(_KUHN_PERMS):
        off = np.zeros(3, dtype=np.int64)
        corners = [off.copy()]
        for ax in perm:
            off[ax] += 1
            corners.append(off.copy())
        for v, c in enumerate(corners):
            p = hi_ + c
            tets[:, t, v] = nid(p[:, 0], p[:, 1], p[:, 2])
    return xyz, tets.reshape(-1, 4).astype(np.int32)


def centroids(xyz: np.ndarray, tets: np.ndarray) -> np.ndarray:
    return xyz[tets].mean(axis=1)


def _in_box(c: np.ndarray, box) -> np.ndarray:
    (x0, x1), (y0, y1), (z0, z1) = box
    return ((c[:, 0] >= x0) & (c[:, 0] <= x1) & (c[:, 1] >= y0) & (c[:, 1] <= y1)
            & (c[:, 2] >= z0) & (c[:, 2] <= z1))


def marine_sigma(cent: np.ndarray, reservoir_box, sigma_res: float,
                 sigma_sea: float = 3.3, sigma_sed: float = 1.0) -> np.ndarray:
    """Sea water above z = 0, sediments below, a resistive reservoir box."""
    s = np.where(cent[:, 2] > 0.0, sigma_sea, sigma_sed).astype(np.float64)
    s[_in_box(cent, reservoir_box)] = sigma_res
    return s


# --------------------------------------------------------------------------
# The five workloads. Config numbering follows the benchmark definitions:
#   1 tiny block model, 2 marine layered, 3 batched multi-RHS on a finer mesh,
#   4 uneven batch of 48 models, 5 learned-initial-guess samples.
# --------------------------------------------------------------------------

def config1(seed: int = 1, n: int = 8) -> Model:
    """[-1000,1000]^3 at n=8 (h=250 m); sigma 1 S/m with a 0.01 S/m block
    [-200,200]x[-200,200]x[-100,0]; x-dipole at (0,0,300), 2 Hz; 20 receivers
    at x=-950..950 (100 m), y=0, z=50."""
    xyz, tets = kuhn_mesh(n, -1000.0, 1000.0, seed)
    c = centroids(xyz, tets)
    sigma = np.ones(len(tets))
    sigma[_in_box(c, ((-200, 200), (-200, 200), (-100, 0)))] = 0.01
    rx = np.stack([-950.0 + 100.0 * np.arange(20), np.zeros(20), np.full(20, 50.0)], 1)
    return Model("cfg1", xyz, tets, sigma, 1.0,
                 [Dipole((0.0, 0.0, 300.0), 2.0)], rx, n, (-1000.0, 1000.0))


def marine_receivers_101() -> np.ndarray:
    return np.stack([-4000.0 + 80.0 * np.arange(101), np.zeros(101),
                     np.full(101, 10.0)], 1)


def config2(seed: int = 2, n: int = 40) -> Model:
    """[-5000,5000]^3 at n=40 (h=250 m); sea 3.3 (z>0), sediments 1 (z<=0),
    reservoir [-1000,1000]^2 x [-1100,-1000] at 0.01; x-dipole at (0,0,50),
    1 Hz; background 3.3 (the conductivity at the source); 101 receivers at
    x=-4000..4000 (80 m), y=0, z=10."""
    xyz, tets = kuhn_mesh(n, -5000.0, 5000.0, seed)
    sigma = marine_sigma(centroids(xyz, tets),
                         ((-1000, 1000), (-1000, 1000), (-1100, -1000)), 0.01)
    return Model("cfg2", xyz, tets, sigma, 3.3,
                 [Dipole((0.0, 0.0, 50.0), 1.0)], marine_receivers_101(),
                 n, (-5000.0, 5000.0))


CFG3_FREQS = (0.25, 0.5, 1.25)


def config3(seed: int = 3, n: int = 100, n_pos: int = 32,
            freqs=CFG3_FREQS) -> Model:
    """The config-2 model at n=100 (h=100 m); 32 x-dipoles at
    x=-3100+200i, y=0, z=50, each at 0.25, 0.5 and 1.25 Hz (96 sources,
    frequency-major order)."""
    xyz, tets = kuhn_mesh(n, -5000.0, 5000.0, seed)
    sigma = marine_sigma(centroids(xyz, tets),
                         ((-1000, 1000), (-1000, 1000), (-1100, -1000)), 0.01)
    srcs = [Dipole((-3100.0 + 200.0 * i, 0.0, 50.0), f)
            for f in freqs for i in range(n_pos)]
    return Model("cfg3", xyz, tets, sigma, 3.3, srcs, marine_receivers_101(),
                 n, (-5000.0, 5000.0))


def layered_marine(n: int = 8, seed: int = 21, lo: float = -1000.0, hi: float = 1000.0,
                   reservoir=((-300.0, 300.0), (-300.0, 300.0), (-250.0, -100.0)), sigma_res: float = 0.02,
                   src=(0.0, 0.0, 60.0), freq: float = 1.0, direction=(1.0, 0.0, 0.0)) -> Model:
    """A marine model for the layered primary field: sea 3.3 S/m above a flat
    sea floor at z = 0 (its nodes are not jittered in z), sediments 1 S/m
    below, a resistive block; the primary field is that of the two
    half-spaces, so dsigma is non-zero in the block only. Receivers on the
    line x = -0.9 ... 0.9 (hi - lo) / 2, y = 0, z = 10 m."""
    xyz, tets = kuhn_mesh(n, lo, hi, seed, flat_z=(0.0,))
    sigma = marine_sigma(centroids(xyz, tets), reservoir, sigma_res)
    L = 0.45 * (hi - lo)
    rx = np.stack([np.linspace(-L, L, 21), np.zeros(21), np.full(21, 10.0)], 1)
    return Model(f"layered-n{n}", xyz, tets, sigma, 3.3, [Dipole(tuple(src), freq, tuple(direction))], rx, n,
                 (lo, hi), layers=(0.0, 3.3, 1.0))


def config4_model(seed: int) -> Model:
    """One model of the uneven batch (seeds 4000..4047).

    Mesh size log-uniform in [1e4, 2e6] tetrahedra -> n = max(12, round((N/6)^(1/3)));
    the config-2 box and layering; reservoir sigma log-uniform in [0.005, 0.05],
    thickness U(50, 300), top depth U(500, 2500) below the sea floor, square side
    U(1000, 4000), centre x, y U(-1500, 1500); f U(0.1, 2); one x-dipole at
    (U(-1000, 1000), 0, 50); 41 receivers from -4000 to 4000 m at z=10."""
    rng = np.random.default_rng([seed, 7])
    n_tets = float(np.exp(rng.uniform(np.log(1e4), np.log(2e6))))
    n = max(12, int(round((n_tets / 6.0) ** (1.0 / 3.0))))
    s_res = float(np.exp(rng.uniform(np.log(0.005), np.log(0.05))))
    thick = float(rng.uniform(50.0, 300.0))
    top = -float(rng.uniform(500.0, 2500.0))
    side = float(rng.uniform(1000.0, 4000.0))
    cx, cy = rng.uniform(-1500.0, 1500.0, size=2)
    f = float(rng.uniform(0.1, 2.0))
    xs = float(rng.uniform(-1000.0, 1000.0))
    xyz, tets = kuhn_mesh(n, -5000.0, 5000.0, seed)
    box = ((cx - side / 2, cx + side / 2), (cy - side / 2, cy + side / 2),
           (top - thick, top))
    sigma = marine_sigma(centroids(xyz, tets), box, s_res)
    rx = np.stack([np.linspace(-4000.0, 4000.0, 41), np.zeros(41), np.full(41, 10.0)], 1)
    return Model(f"cfg4-{seed}", xyz, tets, sigma, 3.3, [Dipole((xs, 0.0, 50.0), f)],
                 rx, n, (-5000.0, 5000.0),
                 meta=dict(sigma_res=s_res, thick=thick, top=top, side=side,
                           centre=(float(cx), float(cy))))


def config4(n_models: int = 48, first_seed: int = 4000) -> List[Model]:
    return [config4_model(first_seed + i) for i in range(n_models)]


CFG5_TRAIN_SEEDS = range(10000, 12000)
CFG5_TEST_SEEDS = range(20000, 20200)


def config5_params(seed: int) -> dict:
    """Random reservoir, source and frequency of one learned-guess sample:
    sigma log-uniform [0.005, 0.05], thickness U(50, 300), top z U(-600, -50),
    square side U(200, 800), centre x, y U(-400, 400), dipole x U(-300, 300),
    z U(150, 400), f U(0.1, 2)."""
    rng = np.random.default_rng([seed, 5])
    s_res = float(np.exp(rng.uniform(np.log(0.005), np.log(0.05))))
    thick = float(rng.uniform(50.0, 300.0))
    top = float(rng.uniform(-600.0, -50.0))
    side = float(rng.uniform(200.0, 800.0))
    cx, cy = (float(v) for v in rng.uniform(-400.0, 400.0, size=2))
    xs = float(rng.uniform(-300.0, 300.0))
    zs = float(rng.uniform(150.0, 400.0))
    f = float(rng.uniform(0.1, 2.0))
    return dict(sigma_res=s_res, thick=thick, top=top, side=side, centre=(cx, cy),
                src=(xs, 0.0, zs), freq=f)


def config5_sample(seed: int, mesh: Optional[Tuple[np.ndarray, np.ndarray]] = None) -> Model:
    """A config-1-sized model (the config-1 mesh, seed 1) with a random reservoir."""
    if mesh is None:
        mesh = kuhn_mesh(8, -1000.0, 1000.0, 1)
    xyz, tets = mesh
    p = config5_params(seed)
    cx, cy = p["centre"]
    hs = p["side"] / 2
    box = ((cx - hs, cx + hs), (cy - hs, cy + hs), (p["top"] - p["thick"], p["top"]))
    sigma = np.ones(len(tets))
    sigma[_in_box(centroids(xyz, tets), box)] = p["sigma_res"]
    rx = np.stack([-950.0 + 100.0 * np.arange(20), np.zeros(20), np.full(20, 50.0)], 1)
    return Model(f"cfg5-{seed}", xyz, tets, sigma, 1.0, [Dipole(p["src"], p["freq"])],
                 rx, 8, (-1000.0, 1000.0), meta=p)


def make_config(i: int, **kw):
    return {1: config1, 2: config2, 3: config3, 4: config4}[i](**kw)
