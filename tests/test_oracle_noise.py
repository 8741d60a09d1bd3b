"""Pins for the oracle's noise generator (CPU only).

The Philox words are checked against numpy's own Philox4x64 implementation
(an independent, published-definition reference available offline); the
normal transform against numpy's log/sin/cos and against the normal law;
the lumped noise against its covariance M_L (eq. wh_def with R = M_L^{1/2}).
"""

import numpy as np
import pytest
from scipy import stats

from oracle import mesh, noise
from workloads import lattice


def test_philox_vector_matches_integer_reference():
    rng = np.random.default_rng(1)
    ctr = rng.integers(0, 2**63, size=64, dtype=np.int64).astype(np.uint64)
    k0, k1 = 0x0123456789ABCDEF, 0xFEDCBA9876543210
    v = noise.philox4x64_10(ctr, k0, k1)
    for i in range(ctr.size):
        ref = noise.philox4x64_10_int([int(ctr[i]), 0, 0, 0], [k0, k1])
        assert [int(w[i]) for w in v] == ref


@pytest.mark.parametrize("key", [(0, 0), (5, 7), (2**64 - 1, 12345)])
def test_philox_matches_numpy_bitgenerator(key):
    # numpy's Philox advances its counter before producing a block, so its
    # first block for counter c-1 is our block for counter c.
    for c in (1, 2, 1000, 2**40):
        bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                              counter=np.array([c - 1, 0, 0, 0], dtype=np.uint64))
        ref = [int(x) for x in bg.random_raw(4)]
        ours = [int(w[0]) for w in noise.philox4x64_10(np.array([c], dtype=np.uint64), *key)]
        assert ours == ref


def test_uniform53_range():
    x = np.array([0, 1 << 11, 2**64 - 1], dtype=np.uint64)
    u = noise.uniform53(x)
    assert u[0] == 0.0 and u[1] == 2.0 ** -53 and u[2] == 1.0 - 2.0 ** -53


def test_log_against_numpy():
    rng = np.random.default_rng(2)
    x = np.concatenate([rng.random(200000), 2.0 ** -rng.uniform(0, 53, 20000),
                        [2.0 ** -53, 0.5, 1.0, np.nextafter(1.0, 0.0), 0.7071067811865476]])
    x = x[x > 0]
    ref = np.log(x)
    got = noise.log_fixed(x)
    assert got[x == 1.0].tolist() == [0.0]
    err = np.abs(got - ref)
    # a few ulp of the result, or of ln2 for tiny results near x = 1
    assert np.all(err <= 4 * np.spacing(np.maximum(np.abs(ref), 1e-300)) + 1e-300)


def test_sincos_against_numpy():
    rng = np.random.default_rng(3)
    u = np.concatenate([rng.random(200000), np.arange(8) / 8.0, np.arange(8) / 8.0 + 2.0 ** -53])
    sn, cs = noise.sincos_2pi_fixed(u)
    assert np.max(np.abs(sn - np.sin(2 * np.pi * u))) < 2e-15
    assert np.max(np.abs(cs - np.cos(2 * np.pi * u))) < 2e-15
    assert np.max(np.abs(sn * sn + cs * cs - 1.0)) < 1e-15
    s0, c0 = noise.sincos_2pi_fixed(np.array([0.0, 0.25, 0.5, 0.75]))
    assert s0[0] == 0.0 and c0[0] == 1.0
    assert s0[1] == 1.0 and abs(c0[1]) < 1e-16
    assert abs(s0[2]) < 1e-16 and c0[2] == -1.0
    assert s0[3] == -1.0 and abs(c0[3]) < 1e-16


def test_normals_are_standard_normal():
    z = np.concatenate([noise.normals(7, s, 100003) for s in range(4)])
    assert abs(z.mean()) < 5 * (1 / np.sqrt(z.size))
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / z.size)
    assert abs(stats.skew(z)) < 5 * np.sqrt(6 / z.size)
    assert abs(stats.kurtosis(z)) < 5 * np.sqrt(24 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # the four components of a block are mutually uncorrelated
    b = noise.normals(7, 0, 400000).reshape(-1, 4)
    c = np.corrcoef(b.T)
    assert np.max(np.abs(c - np.eye(4))) < 5 / np.sqrt(b.shape[0])


def test_normals_keyed_by_seed_and_sample():
    a = noise.normals(0, 0, 1000)
    assert np.array_equal(a, noise.normals(0, 0, 1000))
    assert np.array_equal(a[:37], noise.normals(0, 0, 37))  # prefix-stable
    assert not np.array_equal(a, noise.normals(0, 1, 1000))
    assert not np.array_equal(a, noise.normals(1, 0, 1000))


def test_white_noise_covariance_is_lumped_mass():
    g = lattice(2, 2, lengths=(0.5, 1.5), seed=3)
    m = mesh.build_mesh(g.n_vertices, g.edges, g.lengths, 0.25, "round")
    ML = mesh.lumped_mass(m)
    W = noise.white_noise(ML, 11, 20000)
    var = W.var(axis=0)
    # relative standard error of a variance estimate is sqrt(2/S)
    assert np.all(np.abs(var / ML - 1) < 5 * np.sqrt(2 / W.shape[0]))
    off = np.corrcoef(W.T)[np.triu_indices(ML.size, 1)]
    assert np.max(np.abs(off)) < 5 / np.sqrt(W.shape[0])
    # sample_offset addresses the same stream
    assert np.array_equal(noise.white_noise(ML, 11, 3, sample_offset=5), W[5:8])


# ---- consistent-mass noise (element factors; Phase 2 consistent case, eq. wh_def) ----


def _ragged_mesh(rule="round"):
    """Edges of 1..many elements, a multi-edge, a self-loop and a pendant vertex."""
    edges = np.array([[0, 1], [1, 2], [2, 0], [0, 1], [3, 3], [2, 3], [3, 4]])
    lengths = np.array([0.9, 0.13, 0.41, 0.27, 0.8, 0.05, 0.33])
    return mesh.build_mesh(5, edges, lengths, 0.1, rule)


def test_philox_second_counter_word():
    c = np.arange(9, dtype=np.uint64)
    got = noise.philox4x64_10(c, 77, 5, ctr1=1)
    for i in range(9):
        ref = noise.philox4x64_10_int([i, 1, 0, 0], [77, 5])
        assert [int(w[i]) for w in got] == ref
    # numpy's own Philox (it advances the counter before a block, carrying into word 1)
    for i in (1, 2, 8):
        bg = np.random.Philox(key=np.array([77, 5], dtype=np.uint64),
                              counter=np.array([i - 1, 1, 0, 0], dtype=np.uint64))
        assert [int(x) for x in bg.random_raw(4)] == [int(w[i]) for w in got]
    # the element stream is not the DOF stream
    assert not np.array_equal(got[0], noise.philox4x64_10(c, 77, 5)[0])


@pytest.mark.parametrize("rule", ["round", "ceil"])
def test_consistent_factor_reproduces_consistent_mass(rule):
    m = _ragged_mesh(rule)
    R = noise.consistent_noise_factor(m)
    M = mesh.consistent_mass(m).toarray()
    RRt = (R @ R.T).toarray()
    assert np.abs(RRt - M).max() <= 1e-15 * np.abs(M).max()
    # one element by hand: h = 0.6 gives a^2 + c^2 = 0.2 and a^2 - c^2 = 0.1 = (h/6)[2, 1]
    a, c = noise.element_factor_coefficients(np.array([0.6]))
    assert abs(a[0] ** 2 + c[0] ** 2 - 0.2) < 1e-16 and abs(a[0] ** 2 - c[0] ** 2 - 0.1) < 1e-16


def test_consistent_noise_is_the_factor_times_the_element_draws():
    m = _ragged_mesh()
    R = noise.consistent_noise_factor(m)
    n_el = R.shape[1] // 2
    W = noise.consistent_white_noise(m, 4, 3, sample_offset=2)
    for s in range(3):
        p, q = noise.element_normals(4, 2 + s, n_el)
        xi = np.stack([p, q], axis=1).reshape(-1)
        assert np.abs(R @ xi - W[s]).max() <= 1e-15 * np.abs(W[s]).max()
    assert np.array_equal(noise.consistent_white_noise(m, 4, 1, sample_offset=3), W[1:2])


def test_consistent_noise_covariance_is_consistent_mass():
    g = lattice(2, 2, lengths=(0.5, 1.5), seed=3)
    m = mesh.build_mesh(g.n_vertices, g.edges, g.lengths, 0.25, "round")
    M = mesh.consistent_mass(m).toarray()
    S = 20000
    W = noise.consistent_white_noise(m, 12, S)
    C = W.T @ W / S  # zero mean
    d = np.diag(M)
    se = np.sqrt((np.outer(d, d) + M ** 2) / S)  # standard error of each covariance entry
    assert np.all(np.abs(C - M) < 5 * se)
    # the couplings are seen: every nonzero off-diagonal entry is resolved by its estimate
    nz = (M != 0) & ~np.eye(M.shape[0], dtype=bool)
    assert np.all(M[nz] > 5 * se[nz])
