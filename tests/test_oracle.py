"""Pins of the FP64 oracle against facts that do not come from the oracle.

  hand cases      two single-edge fluxes worked out by hand (golden fixture)
  consistency     F(q, q, n) equals the physical Euler flux from primitives
  symmetries      antisymmetry, degree-1 homogeneity, rotation equivariance
  uniform state   zero residual when the dual cells close (mesh closure)
  conservation    the residual sums to zero over the periodic mesh
  invariance      edge orientation flips and relabelling of nodes and edges
  brute force     residual = signed incidence matrix^T (per-edge fluxes)
  RK scheme       amplification polynomial of the 5-stage scheme on a linear
                  problem; first- and second-order consistency
  stability       a smooth perturbation decays under the negative-sign update
  reductions      compensated sum of squares equals the exactly rounded sum
  derivatives     JVP vs central differences; adjoint vs JVP (dot product)
"""
import math

import numpy as np
import pytest

import meshgen
import oracle
from tests.golden.load import flux_hand_cases, unit_tet_dual

GAMMA = 1.4


def euler_flux_from_primitives(rho, u, p, phi, n):
    """Physical flux of the Euler equations with a passive scalar, f(W).n,
    written from primitive variables."""
    un = float(np.dot(u, n))
    E = p / (GAMMA - 1.0) / rho + 0.5 * float(np.dot(u, u))
    return np.array([rho * un,
                     rho * u[0] * un + p * n[0],
                     rho * u[1] * un + p * n[1],
                     rho * u[2] * un + p * n[2],
                     (rho * E + p) * un,
                     rho * phi * un])


def physical_flux(q, n):
    rho = q[0]
    u = q[1:4] / rho
    p = (GAMMA - 1.0) * (q[4] - 0.5 * rho * float(u @ u))
    return euler_flux_from_primitives(rho, u, p, q[5] / rho, n)


def cons(rho, u, p, phi):
    u = np.asarray(u, float)
    return np.array([rho, rho * u[0], rho * u[1], rho * u[2],
                     p / (GAMMA - 1.0) + 0.5 * rho * float(u @ u), rho * phi])


def random_state(rng):
    return cons(rng.uniform(0.9, 1.1), rng.uniform(-0.3, 0.3, 3), rng.uniform(0.9, 1.1),
                rng.uniform(0, 1))


@pytest.mark.parametrize("case", flux_hand_cases(), ids=lambda c: c[0])
def test_hand_cases(case):
    _, qi, qj, n, F = case
    got = oracle.flux(qi, qj, n)
    assert np.abs(got - F).max() <= 1e-14 * np.abs(F).max()
    # the same edge through the loop: +F at the first node, -F at the second, bitwise
    q = np.stack([qi, qj], axis=1)
    res = oracle.residual(np.array([[0, 1]], np.int32), q, n.reshape(3, 1))
    assert np.array_equal(res[:, 0], got)
    assert np.array_equal(res[:, 1], -got)
    # a 1-based map is not accepted by the 0-based oracle
    with pytest.raises(RuntimeError):
        oracle.residual(np.array([[1, 2]], np.int32), q, n.reshape(3, 1))


def test_flux_symmetries():
    rng = np.random.default_rng(11)
    for _ in range(200):
        qi, qj = random_state(rng), random_state(rng)
        n = rng.normal(size=3)
        F = oracle.flux(qi, qj, n)
        sc = np.abs(F).max() + np.abs(qi).max() * np.linalg.norm(n)
        # consistency with the physical flux
        rho, u, p, phi = qi[0], qi[1:4] / qi[0], None, qi[5] / qi[0]
        p = (GAMMA - 1.0) * (qi[4] - 0.5 * rho * float(u @ u))
        f = euler_flux_from_primitives(rho, u, p, phi, n)
        assert np.abs(oracle.flux(qi, qi, n) - f).max() <= 1e-14 * sc
        # antisymmetry: the flux from j to i across -n is -F
        assert np.abs(oracle.flux(qj, qi, -n) + F).max() <= 1e-14 * sc
        # degree-1 homogeneity in the weight
        s = rng.uniform(0.1, 10.0)
        assert np.abs(oracle.flux(qi, qj, s * n) - s * F).max() <= 1e-14 * s * sc
        # rotation equivariance of the momentum components
        R, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        Rq = lambda q: np.concatenate([q[:1], R @ q[1:4], q[4:]])
        FR = oracle.flux(Rq(qi), Rq(qj), R @ n)
        assert np.abs(FR - Rq(F)).max() <= 1e-14 * sc


@pytest.fixture(scope="module")
def mesh_a():
    return meshgen.config_mesh("A")


@pytest.fixture(scope="module")
def mesh_j():
    return meshgen.build_mesh(8, 1, 0.25)


def test_uniform_state_zero_residual(mesh_a, mesh_j):
    for m in (mesh_a, mesh_j):
        q = np.repeat(cons(1.05, [0.2, -0.1, 0.25], 0.95, 0.4)[:, None], m.N, axis=1)
        res, S = oracle.residual(m.e2n, q, m.w, with_scale=True)
        assert np.all(np.abs(res) <= 1e-13 * S)


def test_conservation(mesh_a, mesh_j):
    for m in (mesh_a, mesh_j):
        q = meshgen.state(m.N, m.perm)
        res, S = oracle.residual(m.e2n, q, m.w, with_scale=True)
        assert np.all(np.abs(res.sum(axis=1)) <= 1e-13 * S.sum(axis=1))
        assert np.abs(res).max() > 1e-6  # a random state is far from steady


def test_orientation_and_relabelling(mesh_j):
    m = mesh_j
    q = meshgen.state(m.N, m.perm)
    res = oracle.residual(m.e2n, q, m.w)
    rng = np.random.default_rng(5)
    flip = rng.random(m.E) < 0.5
    e2n = m.e2n.copy()
    e2n[flip] = e2n[flip][:, ::-1]
    w = m.w.copy()
    w[:, flip] *= -1.0
    res_f = oracle.residual(e2n, q, w)
    scale = np.abs(res).max(axis=1, keepdims=True)
    assert np.abs(res_f - res).max() <= 1e-14 * scale.max()
    # relabel nodes by sigma and shuffle edges: the residual is relabelled
    sigma = rng.permutation(m.N).astype(np.int32)
    order = rng.permutation(m.E)
    q2 = np.empty_like(q)
    q2[:, sigma] = q
    res2 = oracle.residual(sigma[m.e2n[order]], q2, m.w[:, order])
    assert np.abs(res2[:, sigma] - res).max() <= 1e-14 * scale.max()


def test_brute_force_incidence():
    m = meshgen.build_mesh(3, 0, 0.2)
    q = meshgen.state(m.N, m.perm)
    B = np.zeros((m.E, m.N))
    B[np.arange(m.E), m.e2n[:, 0]] = 1.0
    B[np.arange(m.E), m.e2n[:, 1]] = -1.0
    Fe = np.stack([oracle.flux(q[:, i], q[:, j], m.w[:, e]) for e, (i, j) in enumerate(m.e2n)])
    ref = (B.T @ Fe).T
    res = oracle.residual(m.e2n, q, m.w)
    assert np.abs(res - ref).max() <= 1e-14 * np.abs(Fe).max() * 14


def test_rk_amplification_polynomial():
    """On a uniform lattice with uniform density, velocity and pressure the
    scalar component evolves linearly, res_5 = M q_5 (other components stay
    uniform because the dual cells close).  One iteration must then equal
    P(dt M / vol) q_5 with P the scheme's amplification polynomial, which is
    first- and second-order consistent with exp(-X)."""
    m = meshgen.build_mesh(4, 0, 0.0)
    base = cons(1.0, [0.3, 0.1, -0.2], 1.0, 0.0)
    rng = np.random.default_rng(2)
    q = np.repeat(base[:, None], m.N, axis=1)
    q[5] = rng.uniform(0, 1, m.N)
    # M by columns: residual of unit scalar perturbations (linear in q_5)
    M = np.zeros((m.N, m.N))
    for k in range(m.N):
        qk = np.repeat(base[:, None], m.N, axis=1)
        qk[5, k] = 1.0
        M[:, k] = oracle.residual(m.e2n, qk, m.w)[5]
    assert np.abs(M @ q[5] - oracle.residual(m.e2n, q, m.w)[5]).max() < 1e-14
    vol = m.vol[0]
    dt = oracle.dt(m.e2n, q, m.w, m.vol)
    X = dt * M / vol
    # Amplification polynomial of the low-storage 5-stage scheme with stage
    # coefficients (1/4, 1/6, 3/8, 1/2, 1) (Jameson, Schmidt and Turkel 1981):
    # P(X) = 1 - X + X^2/2 - 3 X^3/16 + X^4/32 - X^5/128, written out here so
    # that the oracle's coefficient table and stage order are both checked.
    c = [1.0, 1.0, 1.0 / 2.0, 3.0 / 16.0, 1.0 / 32.0, 1.0 / 128.0]
    # consistency of the scheme: matches exp(-X) to second order
    assert c[1] == 1.0 and c[2] == 0.5
    Pq = np.zeros(m.N)
    Xp = q[5].copy()
    for j in range(6):
        Pq += (-1) ** j * c[j] * Xp
        Xp = X @ Xp
    qn, _ = oracle.rk_iteration(m.e2n, q, m.w, m.vol, dt)
    assert np.abs(qn[5] - Pq).max() <= 1e-14
    assert np.abs(qn[:5] - base[:5, None]).max() <= 1e-15


def test_update_sign_damps_smooth_perturbation(mesh_a):
    m = mesh_a
    base = cons(1.0, [0.2, 0.1, 0.0], 1.0, 0.5)
    pert = 1e-3 * np.sin(2 * np.pi * m.xyz[0])
    q = base[:, None] + pert[None, :] * np.abs(base[:, None]).clip(0.1)
    dt = oracle.dt(m.e2n, q, m.w, m.vol)
    mean0 = q.mean(axis=1, keepdims=True)
    v0 = ((q - mean0) ** 2).sum()
    q1, ss = oracle.rk_iteration(m.e2n, q, m.w, m.vol, dt)
    v1 = ((q1 - q1.mean(axis=1, keepdims=True)) ** 2).sum()
    assert v1 < v0
    # the uniform state is a steady state of the iteration
    qu = np.repeat(base[:, None], m.N, axis=1)
    qu1, _ = oracle.rk_iteration(m.e2n, qu, m.w, m.vol, dt)
    assert np.abs(qu1 - qu).max() <= 1e-14


def test_rk_stage_and_sum_of_squares():
    rng = np.random.default_rng(4)
    N = 5000
    q0 = rng.normal(size=(6, N))
    res = rng.normal(size=(6, N)) * np.exp(rng.uniform(-20, 20, size=(6, N)))
    vol = rng.uniform(0.5, 2.0, N)
    r0 = res.copy()
    q, ss = oracle.rk_stage(q0, res, vol, 0.125)
    assert np.all(res == 0.0)
    for v in range(6):
        exact = math.fsum((r0[v] * r0[v]).tolist())
        assert abs(ss[v] - exact) <= 2 ** -52 * exact
    # the update moves q against the residual
    assert np.all(np.sign(q - q0) == -np.sign(r0)[...] * (r0 != 0))


def test_dt_closed_form_at_rest(mesh_j):
    m = mesh_j
    rho, p = 1.2, 0.9
    q = np.repeat(cons(rho, [0, 0, 0], p, 0.3)[:, None], m.N, axis=1)
    c = math.sqrt(GAMMA * p / rho)
    nn = np.linalg.norm(m.w, axis=0)
    ssum = np.zeros(m.N)
    np.add.at(ssum, m.e2n[:, 0], nn)
    np.add.at(ssum, m.e2n[:, 1], nn)
    expect = 0.5 * np.min(m.vol / (c * ssum))
    assert oracle.dt(m.e2n, q, m.w, m.vol) == pytest.approx(expect, rel=1e-13)
    # hand cases: lambda = 2.5 at both ends, with u.n > 0 (case 1) and u.n < 0
    # (case 2, where |1/2 (U_i + U_j)| = 0.5 only through the absolute value)
    for case in flux_hand_cases():
        _, qi, qj, n, _ = case
        ls = oracle.spectral_radius(np.array([[0, 1]], np.int32), np.stack([qi, qj], 1),
                                    n.reshape(3, 1))
        np.testing.assert_allclose(ls, [2.5, 2.5], rtol=1e-15)


def test_spectral_radius_is_the_flux_dissipation():
    """lambda_e is the coefficient of the flux's dissipation: the density
    component of F is 1/2 (rho_i U_i + rho_j U_j) - 1/2 lambda (rho_j - rho_i),
    so lambda follows from the (hand-pinned) flux and the mass fluxes, for
    random states and weights with u.n of either sign."""
    rng = np.random.default_rng(1403)
    m = 400
    q = np.empty((6, 2 * m))
    n = rng.normal(size=(3, m))
    for k in range(2 * m):
        q[:, k] = random_state(rng)
    e2n = np.arange(2 * m, dtype=np.int32).reshape(m, 2)  # disjoint edges (2k, 2k+1)
    ls = oracle.spectral_radius(e2n, q, n)
    np.testing.assert_array_equal(ls[0::2], ls[1::2])
    signs = []
    for k in range(m):
        qi, qj, nk = q[:, 2 * k], q[:, 2 * k + 1], n[:, k]
        F = oracle.flux(qi, qj, nk)
        Ui, Uj = qi[1:4] @ nk / qi[0], qj[1:4] @ nk / qj[0]
        signs.append(np.sign(Ui + Uj))
        lam = (qi[0] * Ui + qj[0] * Uj - 2.0 * F[0]) / (qj[0] - qi[0])
        scale = (abs(qi[0] * Ui) + abs(qj[0] * Uj) + abs(F[0])) / abs(qj[0] - qi[0])
        assert abs(ls[2 * k] - lam) <= 1e-13 * max(scale, lam), k
    assert min(signs) < 0 < max(signs)


def test_local_dt_closed_form_at_rest(mesh_j):
    """At rest lambda_e = c |n_e|, so each node's step is cfl vol_i / (c sum |n_e|);
    the global step is their minimum."""
    m = mesh_j
    rho, p = 0.8, 1.3
    q = np.repeat(cons(rho, [0, 0, 0], p, -0.2)[:, None], m.N, axis=1)
    c = math.sqrt(GAMMA * p / rho)
    nn = np.linalg.norm(m.w, axis=0)
    ssum = np.zeros(m.N)
    np.add.at(ssum, m.e2n[:, 0], nn)
    np.add.at(ssum, m.e2n[:, 1], nn)
    dtl = oracle.local_dt(m.e2n, q, m.w, m.vol, cfl=0.7)
    np.testing.assert_allclose(dtl, 0.7 * m.vol / (c * ssum), rtol=1e-13)
    assert dtl.min() == pytest.approx(oracle.dt(m.e2n, q, m.w, m.vol, cfl=0.7), rel=1e-15)


def test_local_stage_reduces_to_global_stage():
    rng = np.random.default_rng(6)
    N = 3000
    q0 = rng.normal(size=(6, N))
    res = rng.normal(size=(6, N))
    vol = rng.uniform(0.5, 2.0, N)
    r1, r2 = res.copy(), res.copy()
    qg, ssg = oracle.rk_stage(q0, r1, vol, 0.375 * 0.02)
    ql, ssl = oracle.rk_stage_local(q0, r2, vol, np.full(N, 0.02), 0.375)
    assert np.array_equal(qg, ql) and np.array_equal(ssg, ssl) and np.all(r2 == 0.0)


def test_local_time_stepping_amplification_polynomial():
    """With a step per node the scalar component of the linear problem of
    test_rk_amplification_polynomial advances by P(D M) with D = diag(dt_i /
    vol_i): the same polynomial, now of a non-symmetric matrix, so any slip in
    which node's step scales which residual shows."""
    m = meshgen.build_mesh(4, 0, 0.0)
    base = cons(1.0, [0.3, 0.1, -0.2], 1.0, 0.0)
    rng = np.random.default_rng(12)
    q = np.repeat(base[:, None], m.N, axis=1)
    q[5] = rng.uniform(0, 1, m.N)
    M = np.zeros((m.N, m.N))
    for k in range(m.N):
        qk = np.repeat(base[:, None], m.N, axis=1)
        qk[5, k] = 1.0
        M[:, k] = oracle.residual(m.e2n, qk, m.w)[5]
    dt0 = oracle.dt(m.e2n, q, m.w, m.vol)
    dtl = dt0 * rng.uniform(0.3, 1.0, m.N)
    X = (dtl / m.vol)[:, None] * M
    c = [1.0, 1.0, 1.0 / 2.0, 3.0 / 16.0, 1.0 / 32.0, 1.0 / 128.0]
    Pq = np.zeros(m.N)
    Xp = q[5].copy()
    for j in range(6):
        Pq += (-1) ** j * c[j] * Xp
        Xp = X @ Xp
    qn, _ = oracle.rk_iteration_local(m.e2n, q, m.w, m.vol, dtl)
    assert np.abs(qn[5] - Pq).max() <= 1e-14
    assert np.abs(qn[:5] - base[:5, None]).max() <= 1e-15


def test_gradient_closure_and_linear_exactness(mesh_j):
    """A constant field has zero Green-Gauss sums (closed dual cells); a linear
    field a.x + b gets G_i / vol_i = a exactly at every node none of whose edges
    crosses the periodic boundary (from sum_e n_e (x) d_e = 2 vol I)."""
    m = mesh_j
    q = np.repeat(cons(1.1, [0.2, -0.3, 0.1], 0.8, 0.4)[:, None], m.N, axis=1)
    assert np.abs(oracle.gradient(m.e2n, q, m.w)).max() <= 1e-14 * np.abs(q).max()
    rng = np.random.default_rng(21)
    a = rng.normal(size=(6, 3))
    b = rng.normal(size=6)
    ql = a @ m.xyz + b[:, None]
    G = oracle.gradient(m.e2n, ql, m.w)
    d = m.xyz[:, m.e2n[:, 1]] - m.xyz[:, m.e2n[:, 0]]
    wraps = (np.abs(d) > 0.5).any(axis=0)
    bad = np.zeros(m.N, bool)
    bad[m.e2n[wraps].ravel()] = True
    inner = ~bad
    assert inner.sum() > m.N // 4
    for v in range(6):
        for k in range(3):
            got = G[3 * v + k, inner] / m.vol[inner]
            assert np.abs(got - a[v, k]).max() <= 1e-11 * np.abs(a).max()


def smooth_divergence(m, amp=0.1):
    """div F(q) at the nodes for meshgen.smooth_state: rho(x) varies, velocity
    and pressure are uniform, so each flux component is a multiple of rho'(x)."""
    u = np.array([0.5, 0.2, -0.1])
    drho = amp * 2 * np.pi * np.cos(2 * np.pi * m.xyz[0])
    div = np.zeros((6, m.N))
    div[0] = u[0] * drho                         # (rho u)_x
    div[1:4] = u[:, None] * u[0] * drho[None]    # (rho u_k u)_x, p uniform
    div[4] = 0.5 * (u @ u) * u[0] * drho         # ((rho E + p) u)_x
    div[5] = 0.3 * u[0] * drho                   # (rho phi u)_x
    return div, drho


def test_gradient_and_second_order_flux_convergence():
    """On the regular lattice (h = 1/8, 1/16, 1/32) with a smooth periodic
    state: the Green-Gauss gradient converges at second order, the first-order
    residual / vol approaches div F at first order (the dissipation is O(h)),
    and the reconstructed residual at second order or better."""
    e1, e2, eg = [], [], []
    for n in (8, 16, 32):
        m = meshgen.build_mesh(n, 0, 0.0)
        q = meshgen.smooth_state(m)
        G = oracle.gradient(m.e2n, q, m.w)
        div, drho = smooth_divergence(m)
        r1 = oracle.residual(m.e2n, q, m.w)
        r2 = oracle.residual2(m.e2n, q, G, m.vol, m.w, meshgen.edge_vectors(m))
        e1.append(np.abs(r1 / m.vol - div).max())
        e2.append(np.abs(r2 / m.vol - div).max())
        eg.append(np.abs(G[0] / m.vol - drho).max())
    for k in range(2):
        assert 1.7 < e1[k] / e1[k + 1] < 2.3
        assert e2[k] / e2[k + 1] > 3.5
        assert 3.5 < eg[k] / eg[k + 1] < 4.5
    assert e2[-1] < 0.05 * e1[-1]


def test_second_order_residual_special_cases(mesh_j):
    m = mesh_j
    q = meshgen.state(m.N, m.perm)
    dx = meshgen.edge_vectors(m)
    # zero gradients: exactly the first-order residual
    r2 = oracle.residual2(m.e2n, q, np.zeros((18, m.N)), m.vol, m.w, dx)
    assert np.array_equal(r2, oracle.residual(m.e2n, q, m.w))
    # conservation with gradients
    G = oracle.gradient(m.e2n, q, m.w)
    r2 = oracle.residual2(m.e2n, q, G, m.vol, m.w, dx)
    assert np.abs(r2.sum(axis=1)).max() <= 1e-12 * np.abs(r2).max()
    # a linear profile along one edge with its exact gradient at both ends
    # reconstructs the midpoint state on both sides: no dissipation, the flux is
    # the physical flux of the midpoint state
    _, qi, qj, n, _ = flux_hand_cases()[0]
    d = np.array([0.3, -0.2, 0.5])
    g = np.outer(qj - qi, d) / (d @ d)          # any gradient with g.d = qj - qi
    vol = np.array([2.0, 3.0])
    Gs = np.concatenate([(g * vol[0]).reshape(18, 1), (g * vol[1]).reshape(18, 1)], 1)
    r = oracle.residual2(np.array([[0, 1]], np.int32), np.stack([qi, qj], 1), Gs, vol,
                         n.reshape(3, 1), d.reshape(3, 1))
    qm = 0.5 * (qi + qj)
    np.testing.assert_allclose(r[:, 0], physical_flux(qm, n), rtol=1e-13, atol=1e-14)


def test_geometry_unit_tet_hand_values():
    xyz = np.array([[0.0, 1, 0, 0], [0, 0, 1, 0], [0, 0, 0, 1]])
    t2n = np.array([[0, 1, 2, 3]], np.int32)
    pairs = list(meshgen.TET_LOCAL_EDGES)
    # the map orients edges 1->0 and 2->3 backwards on purpose: signs follow e2n
    e2n = np.array([[1, 0], [0, 2], [0, 3], [1, 2], [1, 3], [3, 2]], np.int32)
    t2e = np.arange(6, dtype=np.int32)[None, :]
    w, vol = oracle.geometry(e2n, t2n, t2e, xyz, period=0.0)
    ref = unit_tet_dual()
    for k, (a, b) in enumerate(pairs):
        sign = 1.0 if (e2n[k, 0], e2n[k, 1]) == (a, b) else -1.0
        np.testing.assert_allclose(24 * w[:, k], sign * ref[(a, b)], atol=1e-15)
    np.testing.assert_allclose(vol, np.full(4, 1.0 / 24.0), rtol=1e-15)


def test_geometry_closure_volume_and_linear_exactness(mesh_j):
    m = mesh_j
    t2n = m.tets()
    t2e = meshgen.tet_edges(m, t2n)
    w, vol = oracle.geometry(m.e2n, t2n, t2e, m.xyz)
    assert vol.sum() == pytest.approx(1.0, rel=1e-13)
    assert vol.min() > 0
    # closed dual cells: the face vectors around every node sum to zero
    S = np.zeros((3, m.N))
    for d in range(3):
        np.add.at(S[d], m.e2n[:, 0], w[d])
        np.add.at(S[d], m.e2n[:, 1], -w[d])
    assert np.abs(S).max() <= 1e-15
    # sum over edges at i of n (x) (x_j - x_i), signed toward i's neighbour, = 2 vol_i I
    dx = meshgen.edge_vectors(m)
    M = np.zeros((3, 3, m.N))
    for a in range(3):
        for b in range(3):
            f = w[a] * dx[b]
            np.add.at(M[a, b], m.e2n[:, 0], f)
            np.add.at(M[a, b], m.e2n[:, 1], f)
    eye = np.eye(3)[:, :, None] * (2 * vol)[None, None, :]
    assert np.abs(M - eye).max() <= 1e-14


def test_geometry_adjoint_central_differences():
    m = meshgen.build_mesh(4, 1, 0.25)
    t2n = m.tets()
    t2e = meshgen.tet_edges(m, t2n)
    rng = np.random.default_rng(31)
    wbar, volbar = rng.normal(size=(3, m.E)), rng.normal(size=m.N)
    xbar = oracle.geometry_adjoint(m.e2n, t2n, t2e, m.xyz, wbar, volbar)

    def J(x):
        w, vol = oracle.geometry(m.e2n, t2n, t2e, x)
        return float((wbar * w).sum() + (volbar * vol).sum())

    for _ in range(3):
        dx = rng.normal(size=(3, m.N)) * 1e-3
        h = 1e-3
        fd = (J(m.xyz + h * dx) - J(m.xyz - h * dx)) / (2 * h)
        assert float((xbar * dx).sum()) == pytest.approx(fd, rel=1e-8, abs=1e-14)


def test_shape_sensitivity_chain_central_differences():
    """dJ/dx for J = rbar . R(q, w(x)) at fixed q: the flux adjoint gives
    wbar = (dR/dw)^T rbar, the geometry adjoint carries it to the nodes."""
    m = meshgen.build_mesh(4, 1, 0.25)
    t2n = m.tets()
    t2e = meshgen.tet_edges(m, t2n)
    q = meshgen.state(m.N, m.perm)
    rng = np.random.default_rng(32)
    rbar = rng.normal(size=(6, m.N))
    w0, _ = oracle.geometry(m.e2n, t2n, t2e, m.xyz)
    _, wbar = oracle.adjoint(m.e2n, q, w0, rbar)
    xbar = oracle.geometry_adjoint(m.e2n, t2n, t2e, m.xyz, wbar, np.zeros(m.N))

    def J(x):
        w, _ = oracle.geometry(m.e2n, t2n, t2e, x)
        return float((rbar * oracle.residual(m.e2n, q, w)).sum())

    dx = rng.normal(size=(3, m.N)) * 1e-3
    h = 1e-3
    fd = (J(m.xyz + h * dx) - J(m.xyz - h * dx)) / (2 * h)
    assert float((xbar * dx).sum()) == pytest.approx(fd, rel=1e-6)


def test_edge_jacobian_vs_central_differences():
    rng = np.random.default_rng(9)
    for _ in range(30):
        qi, qj, n = random_state(rng), random_state(rng), rng.normal(size=3)
        F, J = oracle.edge_jacobian(qi, qj, n)
        assert np.array_equal(F, oracle.flux(qi, qj, n))
        x = np.concatenate([qi, qj, n])
        for k in range(15):
            h = 1e-6 * max(1.0, abs(x[k]))
            xp, xm = x.copy(), x.copy()
            xp[k] += h
            xm[k] -= h
            fd = (oracle.flux(xp[:6], xp[6:12], xp[12:]) -
                  oracle.flux(xm[:6], xm[6:12], xm[12:])) / (2 * h)
            assert np.abs(fd - J[:, k]).max() <= 1e-6 * max(1.0, np.abs(J).max())


def test_jvp_fd_and_adjoint_dot_product(mesh_j):
    m = mesh_j
    q = meshgen.state(m.N, m.perm)
    rng = np.random.default_rng(21)
    dq = rng.normal(size=q.shape)
    dw = rng.normal(size=m.w.shape) * np.linalg.norm(m.w, axis=0)
    jv = oracle.jvp(m.e2n, q, m.w, dq, dw)
    h = 1e-6
    fd = (oracle.residual(m.e2n, q + h * dq, m.w + h * dw) -
          oracle.residual(m.e2n, q - h * dq, m.w - h * dw)) / (2 * h)
    assert np.abs(fd - jv).max() <= 1e-6 * np.abs(jv).max()
    rbar = rng.normal(size=q.shape)
    qbar, wbar = oracle.adjoint(m.e2n, q, m.w, rbar)
    lhs = float((rbar * jv).sum())
    rhs = float((qbar * dq).sum() + (wbar * dw).sum())
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # the residual's value is untouched by the tangent
    assert np.array_equal(oracle.jvp(m.e2n, q, m.w), np.zeros_like(q))
