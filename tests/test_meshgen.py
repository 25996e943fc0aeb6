"""Pins of the seeded input generator: topology, geometry and determinism.

The generator only builds inputs; these checks pin it against facts of the
mesh family itself (Euler characteristic of the 3-torus, closed dual control
volumes, exactness of median-dual weights for linear fields), not against
itself.
"""
import numpy as np
import pytest

import meshgen


def _faces(tets):
    f = np.concatenate([tets[:, [0, 1, 2]], tets[:, [0, 1, 3]], tets[:, [0, 2, 3]],
                        tets[:, [1, 2, 3]]])
    f = np.sort(f, axis=1)
    uniq, counts = np.unique(f, axis=0, return_counts=True)
    return uniq, counts


@pytest.mark.parametrize("n,split,jitter", [(3, 0, 0.0), (4, 0, 0.2), (4, 1, 0.0), (8, 1, 0.25)])
def test_topology_euler_and_counts(n, split, jitter):
    m = meshgen.build_mesh(n, split, jitter)
    N = n ** 3
    assert m.N == N
    six = N if split == 0 else N // 2
    assert m.six_cubes == six
    # every cube is 5 or 6 tets; edges are 3 axis + 3 face diagonals per node + body diagonals
    assert m.T == 5 * N + six
    assert m.E == 6 * N + six
    tets = m.tets()
    assert tets.shape == (m.T, 4)
    uniq, counts = _faces(tets)
    # a closed 3-manifold: every triangle bounds exactly two tets
    assert np.all(counts == 2)
    F = len(uniq)
    assert F == 2 * m.T
    # Euler characteristic of the 3-torus is zero
    assert m.N - m.E + F - m.T == 0
    # the edge list is exactly the set of tet edges
    te = np.concatenate([tets[:, [a, b]] for a in range(4) for b in range(a + 1, 4)])
    te = np.unique(np.sort(te, axis=1), axis=0)
    me = np.unique(np.sort(m.e2n, axis=1), axis=0)
    assert len(me) == m.E
    assert np.array_equal(te, me)


def test_config_edge_counts():
    assert meshgen.sizes(20, 0) == (8000, 56000, 48000)
    assert meshgen.sizes(100, 0) == (1_000_000, 7_000_000, 6_000_000)
    assert meshgen.sizes(160, 1) == (4_096_000, 26_624_000, 22_528_000)
    with pytest.raises(ValueError):
        meshgen.sizes(2, 0)
    with pytest.raises(ValueError):
        meshgen.sizes(6, 1)  # the layered mix needs n % 4 == 0 to close periodically


def test_unit_tet_dual_weights():
    nv, v = meshgen.tet_dual([0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0, 1])
    assert v == pytest.approx(1.0 / 6.0, rel=1e-15)
    expect = np.array([[2, 1, 1], [1, 2, 1], [1, 1, 2], [-1, 1, 0], [-1, 0, 1], [0, -1, 1]]) / 24.0
    np.testing.assert_allclose(nv, expect, rtol=0, atol=1e-17)
    # Inside one tet, vertex v's sub-cell is closed by its three dual faces and
    # one third of each of the three tet faces at v.  Check on random tets too.
    rng = np.random.default_rng(3)
    edges = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    for x in [np.array([0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0, 1], float)] + [
            rng.normal(size=12) for _ in range(20)]:
        X = x.reshape(4, 3)
        if np.linalg.det(np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]])) < 0:
            X[[2, 3]] = X[[3, 2]]
        nv, v = meshgen.tet_dual(X.reshape(-1))
        assert v > 0
        for vtx in range(4):
            dual = sum((+1 if a == vtx else -1) * nv[k]
                       for k, (a, b) in enumerate(edges) if vtx in (a, b))
            outer = np.zeros(3)
            for opp in range(4):  # face opposite vertex `opp`, if it contains vtx
                if opp == vtx:
                    continue
                a, b, c = [k for k in range(4) if k != opp]
                A = 0.5 * np.cross(X[b] - X[a], X[c] - X[a])
                if np.dot(A, X[opp] - X[a]) > 0:
                    A = -A
                outer += A / 3.0
            assert np.abs(dual + outer).max() <= 1e-14 * max(1.0, np.abs(X).max() ** 2)


def _node_sums(m):
    a, b = m.e2n[:, 0], m.e2n[:, 1]
    clos = np.zeros((3, m.N))
    scale = np.zeros(m.N)
    for d in range(3):
        np.add.at(clos[d], a, m.w[d])
        np.add.at(clos[d], b, -m.w[d])
    nn = np.linalg.norm(m.w, axis=0)
    np.add.at(scale, a, nn)
    np.add.at(scale, b, nn)
    return clos, scale, nn


@pytest.mark.parametrize("n,split,jitter", [(20, 0, 0.0), (12, 0, 0.2), (16, 1, 0.25)])
def test_volumes_closure_weights(n, split, jitter):
    m = meshgen.build_mesh(n, split, jitter)
    assert abs(m.vol.sum() - 1.0) < 1e-12
    assert m.vol.min() > 0.0
    clos, scale, nn = _node_sums(m)
    assert np.all(np.abs(clos).max(axis=0) <= 1e-13 * scale)
    assert nn.min() > 0.0
    if jitter == 0.0:
        # uniform Kuhn lattice: every dual volume is h^3
        np.testing.assert_allclose(m.vol, 1.0 / n ** 3, rtol=1e-12)


@pytest.mark.parametrize("n,split,jitter", [(5, 0, 0.2), (8, 1, 0.25)])
def test_linear_exactness(n, split, jitter):
    """Median-dual weights integrate linear fields exactly: for every node,
    sum over incident edges of n_e (x) (x_j - x_i), with n_e oriented out of
    the node, equals 2 vol_i I (Green-Gauss on the closed dual cell)."""
    m = meshgen.build_mesh(n, split, jitter)
    a, b = m.e2n[:, 0], m.e2n[:, 1]
    d = m.xyz[:, b] - m.xyz[:, a]
    d -= np.round(d)  # periodic unwrap; every edge is shorter than half the box
    M = np.zeros((m.N, 3, 3))
    for r in range(3):
        for c in range(3):
            np.add.at(M[:, r, c], a, m.w[r] * d[c])
            np.add.at(M[:, r, c], b, m.w[r] * d[c])
    target = 2.0 * m.vol[:, None, None] * np.eye(3)
    assert np.abs(M - target).max() <= 1e-12 * m.vol.max()


def test_determinism_and_seeds():
    a = meshgen.build_mesh(6, 0, 0.2, seed=5)
    b = meshgen.build_mesh(6, 0, 0.2, seed=5)
    c = meshgen.build_mesh(6, 0, 0.2, seed=6)
    for x, y in [(a.e2n, b.e2n), (a.w, b.w), (a.vol, b.vol), (a.perm, b.perm)]:
        assert x.tobytes() == y.tobytes()
    assert a.perm.tobytes() != c.perm.tobytes()
    assert np.array_equal(np.sort(a.perm), np.arange(a.N))
    q1 = meshgen.state(a.N, a.perm)
    q2 = meshgen.state(a.N, a.perm)
    assert q1.tobytes() == q2.tobytes()
    assert meshgen.normal(11).tobytes() == meshgen.normal(11).tobytes()


def test_state_distribution():
    m = meshgen.build_mesh(10, 0, 0.0)
    q = meshgen.state(m.N, m.perm)
    rho = q[0]
    u = q[1:4] / rho
    p = 0.4 * (q[4] - 0.5 * rho * (u ** 2).sum(0))
    phi = q[5] / rho
    assert rho.min() >= 0.9 and rho.max() < 1.1
    assert np.abs(u).max() <= 0.3
    assert p.min() >= 0.9 - 1e-12 and p.max() < 1.1 + 1e-12
    assert phi.min() >= 0.0 and phi.max() < 1.0
    # the field is drawn in generator order: the same physical field for any labelling
    q0 = meshgen.state(m.N, None)
    np.testing.assert_array_equal(q[:, m.perm], q0)
    z = meshgen.normal(200000)
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1.0) < 0.01


@pytest.mark.slow
def test_large_layered_mesh():
    m = meshgen.config_mesh("E")
    assert (m.N, m.E, m.T) == (4_096_000, 26_624_000, 22_528_000)
    assert m.six_cubes == m.N // 2
    assert m.vol.min() > 0.0
    assert abs(m.vol.sum() - 1.0) < 1e-10


def test_tet_edges_against_a_sorted_key_lookup():
    """The C lookup of each tet's six edges agrees with an independent numpy
    lookup (sorted (min, max) node-pair keys), and every edge is found."""
    for n, split in ((3, 0), (8, 1), (12, 0)):
        m = meshgen.build_mesh(n, split, 0.2)
        t2n = m.tets()
        got = meshgen.tet_edges(m, t2n)
        lo = np.minimum(m.e2n[:, 0], m.e2n[:, 1]).astype(np.int64)
        hi = np.maximum(m.e2n[:, 0], m.e2n[:, 1]).astype(np.int64)
        key = lo * m.N + hi
        order = np.argsort(key)
        for k, (a, b) in enumerate(meshgen.TET_LOCAL_EDGES):
            p, q = t2n[:, a].astype(np.int64), t2n[:, b].astype(np.int64)
            want = np.minimum(p, q) * m.N + np.maximum(p, q)
            pos = np.searchsorted(key[order], want)
            assert np.array_equal(key[order][pos], want)
            assert np.array_equal(order[pos], got[:, k])
    # a tet edge missing from the map is an error, not a wrong answer
    bad = t2n.copy()
    bad[0, 1] = bad[0, 0]
    with pytest.raises(ValueError):
        meshgen.tet_edges(m, bad)
