"""Seeded generators for the metric graphs the sampler is exercised on.

Every generator returns a :class:`Graph` (vertex count, ``[E, 2]`` int64 edge
list oriented ``u -> v``, ``[E]`` float64 edge lengths).  The shapes mirror the
workloads in the paper and in the benchmark configurations:

* lattices (the paper's convergence study defers to lattice-like graphs; the
  throughput configurations use 4x4, 64x64 and 256x256 lattices),
* Barabasi-Albert preferential-attachment graphs (the paper's performance
  study uses BA graphs with attachment parameter 2 and unit lengths, see its
  "Performance comparison" subsection and the two tables that follow it),
* random geometric graphs (training and evaluation graphs for the learned
  preconditioner).

All randomness comes from ``numpy.random.default_rng(seed)``.
"""

from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class Graph:
    n_vertices: int
    edges: np.ndarray  # int64 [E, 2], u -> v
    lengths: np.ndarray  # float64 [E]
    name: str = ""

    @property
    def n_edges(self) -> int:
        return int(self.edges.shape[0])

    def validate(self) -> None:
        e = self.edges
        assert e.dtype == np.int64 and e.ndim == 2 and e.shape[1] == 2
        assert self.lengths.dtype == np.float64 and self.lengths.shape == (e.shape[0],)
        assert e.min(initial=0) >= 0 and e.max(initial=-1) < self.n_vertices
        deg = np.bincount(e.ravel(), minlength=self.n_vertices)
        assert (deg > 0).all(), "isolated vertex"


def _lengths(n: int, lengths, rng) -> np.ndarray:
    if lengths is None:
        return np.ones(n, dtype=np.float64)
    lo, hi = lengths
    return rng.uniform(lo, hi, size=n).astype(np.float64)


def lattice(nx: int, ny: int, lengths=None, seed: int = 0, name: str = "") -> Graph:
    """Rectangular lattice with ``nx`` rows and ``ny`` columns.

    Vertex ``v = i*ny + j``.  Horizontal edges come first in row-major order,
    then vertical edges in row-major order; every edge points from the lower
    to the higher vertex index.  ``lengths=None`` gives unit lengths,
    ``lengths=(lo, hi)`` draws iid Uniform[lo, hi] lengths from ``seed``.
    """
    rng = np.random.default_rng(seed)
    horiz = [(i * ny + j, i * ny + j + 1) for i in range(nx) for j in range(ny - 1)]
    vert = [(i * ny + j, (i + 1) * ny + j) for i in range(nx - 1) for j in range(ny)]
    edges = np.array(horiz + vert, dtype=np.int64).reshape(-1, 2)
    g = Graph(nx * ny, edges, _lengths(edges.shape[0], lengths, rng), name or f"lattice{nx}x{ny}")
    g.validate()
    return g


def interval(length: float = 1.0) -> Graph:
    """A single edge ``0 -> 1`` of the given length."""
    return Graph(2, np.array([[0, 1]], dtype=np.int64), np.array([length], dtype=np.float64), "interval")


def preferential_attachment(n: int, m: int, lengths=None, seed: int = 0, name: str = "") -> Graph:
    """Barabasi-Albert graph: start from a star on ``m+1`` vertices, then attach
    each new vertex to ``m`` distinct existing vertices chosen with probability
    proportional to degree.  ``m(n-m)`` edges; ``m=1`` gives a random tree.
    """
    assert n > m >= 1
    rng = np.random.default_rng(seed)
    edges = [(0, j) for j in range(1, m + 1)]
    # repeated-endpoint list: picking uniformly from it is degree-proportional
    ends = [0] * m + list(range(1, m + 1))
    for v in range(m + 1, n):
        chosen: set[int] = set()
        while len(chosen) < m:
            chosen.add(ends[int(rng.integers(len(ends)))])
        for u in sorted(chosen):
            edges.append((u, v))
            ends.extend((u, v))
    e = np.array(edges, dtype=np.int64)
    g = Graph(n, e, _lengths(e.shape[0], lengths, rng), name or f"ba{n}_m{m}")
    g.validate()
    return g


def random_geometric(n: int, seed: int = 0, mean_degree: float = 4.0, name: str = "") -> Graph:
    """Random geometric graph: ``n`` points uniform in a sqrt(n) x sqrt(n)
    square, an edge between every pair closer than ``r`` with
    ``pi r^2 = mean_degree`` (unit point density), edge length = Euclidean
    distance.  Isolated points are dropped and vertices renumbered.
    """
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(seed)
    side = np.sqrt(n)
    pts = rng.uniform(0.0, side, size=(n, 2))
    r = np.sqrt(mean_degree / np.pi)
    pairs = cKDTree(pts).query_pairs(r, output_type="ndarray").astype(np.int64)
    pairs.sort(axis=1)
    pairs = pairs[np.lexsort((pairs[:, 1], pairs[:, 0]))]
    used = np.unique(pairs.ravel())
    remap = -np.ones(n, dtype=np.int64)
    remap[used] = np.arange(used.size, dtype=np.int64)
    lens = np.linalg.norm(pts[pairs[:, 0]] - pts[pairs[:, 1]], axis=1)
    # a pair at distance 0 would be a degenerate edge; drop it
    keep = lens > 0
    e = remap[pairs[keep]]
    g = Graph(int(used.size), e, lens[keep].astype(np.float64), name or f"rgg{n}")
    used2 = np.unique(e.ravel())
    if used2.size != g.n_vertices:  # only if a zero-length pair isolated a vertex
        remap2 = -np.ones(g.n_vertices, dtype=np.int64)
        remap2[used2] = np.arange(used2.size, dtype=np.int64)
        g = Graph(int(used2.size), remap2[e], g.lengths, g.name)
    g.validate()
    return g


# --------------------------------------------------------------------------
# Benchmark configurations (graph + parameters).  Sizes follow the five
# configurations the throughput study is quoted on; the paper itself only
# fixes the BA performance workload (unit lengths, h = 2^-6).
# --------------------------------------------------------------------------

def config_c1() -> dict:
    """4x4 unit lattice, h = 1/64, kappa = 5, beta = 0.75, step 0.5, 16 samples."""
    return dict(graph=lattice(4, 4), h=1.0 / 64, rule="ceil", kappa=5.0, beta=0.75,
                quad_step=0.5, n_samples=16, seed=0, tol=1e-12)


def config_c2(beta: float = 0.6, n_samples: int = 256) -> dict:
    """64x64 lattice, lengths U[0.5,1.5] (seed 1), h = 1/256 rounded mesh,
    kappa = 10, beta in {0.6, 0.85}, step 0.3, 256 samples."""
    return dict(graph=lattice(64, 64, lengths=(0.5, 1.5), seed=1), h=1.0 / 256, rule="round",
                kappa=10.0, beta=beta, quad_step=0.3, n_samples=n_samples, seed=0, tol=1e-12)


def config_c3(n_graphs: int = 64, seed: int = 3, max_edges: int = 20000) -> dict:
    """64 uneven graphs: half preferential-attachment trees, half near-square
    lattices, edge counts log-uniform in [100, max_edges], lengths U[0.1, 2.0],
    h = 1/128 rounded mesh, kappa_g ~ U[2, 20], beta = 0.75, 32 samples."""
    rng = np.random.default_rng(seed)
    graphs, kappas = [], []
    for gi in range(n_graphs):
        target = int(np.exp(rng.uniform(np.log(100), np.log(max_edges))))
        gseed = int(rng.integers(1 << 31))
        if gi % 2 == 0:
            g = preferential_attachment(target + 1, 1, lengths=(0.1, 2.0), seed=gseed, name=f"tree{gi}")
        else:
            # nx*(ny-1) + (nx-1)*ny ~ 2 nx ny edges for a near-square lattice
            nx = max(2, int(round(np.sqrt(target / 2.0))))
            ny = max(2, int(round(target / (2.0 * nx))))
            g = lattice(nx, ny, lengths=(0.1, 2.0), seed=gseed, name=f"grid{gi}")
        graphs.append(g)
        kappas.append(float(rng.uniform(2.0, 20.0)))
    return dict(graphs=graphs, kappas=kappas, h=1.0 / 128, rule="round", beta=0.75,
                quad_step=None, n_samples=32, seed=0, tol=1e-12)


def config_c4(n_samples: int = 64) -> dict:
    """256x256 lattice, lengths U[0.5,1.5] (seed 4), h = 1/512 rounded mesh,
    kappa = 20, beta = 0.55, step 0.2 with |l| <= 46 (e^{2y} in [1e-8, 1e8])."""
    return dict(graph=lattice(256, 256, lengths=(0.5, 1.5), seed=4), h=1.0 / 512, rule="round",
                kappa=20.0, beta=0.55, quad_step=0.2, k_minus=46, k_plus=46,
                n_samples=n_samples, seed=0, tol=1e-12)


def config_c5_train(n_graphs: int = 16, seed: int = 50) -> list[dict]:
    """Training graphs for the learned preconditioner: random geometric graphs
    with 2k..20k points, mean degree 4, h = 1/256, kappa ~ U[2, 20]."""
    rng = np.random.default_rng(seed)
    out = []
    for gi in range(n_graphs):
        n = int(rng.integers(2000, 20001))
        out.append(dict(graph=random_geometric(n, seed=int(rng.integers(1 << 31)), name=f"rgg_train{gi}"),
                        kappa=float(rng.uniform(2.0, 20.0))))
    return out


def config_c5_eval(n_points: int = 100_000) -> dict:
    """Held-out random geometric graph (~100k points, ~200k edges, seed 5),
    h = 1/256, kappa = 2, beta = 0.75, 64 samples."""
    return dict(graph=random_geometric(n_points, seed=5, name="rgg_eval"), h=1.0 / 256, rule="round",
                kappa=2.0, beta=0.75, quad_step=None, n_samples=64, seed=0, tol=1e-12)


def config_paper_ba(n: int = 50_000) -> dict:
    """The paper's performance workload: BA graph, attachment 2, unit lengths,
    h = 2^-6 (its lumped-vs-consistent tables)."""
    return dict(graph=preferential_attachment(n, 2, seed=7), h=2.0 ** -6, rule="ceil",
                kappa=1.0, beta=0.75, quad_step=None, n_samples=1, seed=0, tol=1e-12)
