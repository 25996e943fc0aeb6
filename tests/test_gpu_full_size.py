"""Parity at the full workload sizes, in the launch configuration bench.py
times (owner variant, Morton renumbering, clusters of 512 nodes), against
the FP64 oracle: whole arrays where the oracle finishes in seconds, sampled
outputs computed one by one where it does not (the adjoint), and properties
that hold at any size for the 100-iteration FP32 trajectory.
"""
import math

import numpy as np
import pytest
import torch

import meshgen
import oracle
import paper_1403_7209_amd as pk
from tests._util import normwise, report

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
BENCH = dict(renumber="morton", block_size=512, cluster_size=512)


@pytest.fixture(scope="module")
def mesh_e():
    print("[building the 160^3 layered mesh]", flush=True)
    m = meshgen.config_mesh("E")
    q = meshgen.state(m.N, m.perm)
    return m, q


@pytest.fixture(scope="module")
def prob_e(mesh_e):
    m, q = mesh_e
    ctx = pk.Context(DEV)
    p64 = pk.FluxProblem(ctx, m.e2n, m.w, m.vol, q, coords=m.xyz, **BENCH)
    p32 = pk.FluxProblem(ctx, m.e2n, m.w, m.vol, q, fp32=True, like=p64)
    return p64, p32


def test_plan_at_full_size(prob_e, mesh_e):
    p64, _ = prob_e
    m, _ = mesh_e
    assert p64.ctx.plan_verify(p64.e2n)["ok"]
    assert p64.info["owner_ok"]
    assert m.E <= p64.info["owner_edge_visits"] <= 1.4 * m.E


def test_fp64_residual_full(prob_e, mesh_e):
    p64, _ = prob_e
    m, q = mesh_e
    print("[E: oracle residual]", flush=True)
    ref = oracle.residual(m.e2n, q, m.w)
    for variant, acc in ((pk.OWNER, pk.WRITE), (pk.OWNER, pk.INC), (pk.COLOURED, pk.INC),
                         (pk.FLAT, pk.INC), (pk.ATOMIC, pk.INC), (pk.COLOURED_LDS_ATOMIC, pk.INC)):
        res = torch.full((6, m.N), 0.0 if acc == pk.INC else 7.0, dtype=torch.float64, device=DEV)
        p64.residual(p64.qa, res, variant, acc)
        p64.ctx.sync()
        assert report(f"E residual v{variant} acc{acc}", normwise(p64.nodes_out(res), ref), 1e-12)


def test_fp32_residual_full(prob_e, mesh_e):
    _, p32 = prob_e
    m, q = mesh_e
    q32 = q.astype(np.float32).astype(np.float64)
    w32 = m.w.astype(np.float32).astype(np.float64)
    ref = oracle.residual(m.e2n, q32, w32)
    res = torch.empty((6, m.N), dtype=torch.float64, device=DEV)
    p32.residual(p32.qa, res, pk.OWNER, pk.WRITE)
    p32.ctx.sync()
    assert report("E fp32 residual", normwise(p32.nodes_out(res), ref), 1e-5)


def test_fp32_fused_stage_full(prob_e, mesh_e):
    """One FP32-storage stage with the update fused into the edge loop (the
    bench's FP32 kernel) against the oracle fed the FP32-rounded inputs."""
    _, p32 = prob_e
    m, q = mesh_e
    q32 = q.astype(np.float32).astype(np.float64)
    w32 = m.w.astype(np.float32).astype(np.float64)
    adt = 0.25 * oracle.dt(m.e2n, q32, w32, m.vol)
    res = oracle.residual(m.e2n, q32, w32)
    q1_ref, ss_ref = oracle.rk_stage(q32, res, m.vol, adt)
    out = torch.empty_like(p32.qa)
    ss = torch.zeros(6, dtype=torch.float64, device=DEV)
    qa = p32.dat(p32.qa, "qa")
    p32.ctx.edge_flux_stage(p32.edges, p32.e2n, qa, p32.w, qa, p32.vol, p32.dat(out, "out"), adt,
                            ss, p32.gamma)
    p32.ctx.sync()
    assert report("E fp32 fused stage state", normwise(p32.nodes_out(out), q1_ref), 1e-5)
    assert report("E fp32 fused stage rms", normwise(np.sqrt(ss.cpu().numpy() / m.N),
                                                     np.sqrt(ss_ref / m.N)), 1e-5)


def test_time_step_and_rk_iteration_full(prob_e, mesh_e):
    p64, _ = prob_e
    m, q = mesh_e
    dt_ref = oracle.dt(m.e2n, q, m.w, m.vol)
    dt = p64.compute_dt(0.5, pk.OWNER)
    assert abs(dt - dt_ref) <= 1e-12 * dt_ref
    print("[E: oracle RK iteration]", flush=True)
    q1, ss = oracle.rk_iteration(m.e2n, q, m.w, m.vol, dt_ref)
    qa0 = p64.qa.clone()
    p64.rk_iteration(dt_ref, pk.OWNER)
    p64.ctx.sync()
    assert report("E state after one iteration", normwise(p64.nodes_out(p64.qa), q1), 1e-12)
    assert report("E stage rms", normwise(p64.rms(), np.sqrt(ss / m.N)), 1e-12)
    p64.qa.copy_(qa0)


def test_local_time_steps_full(prob_e, mesh_e):
    p64, _ = prob_e
    m, q = mesh_e
    ref = oracle.local_dt(m.e2n, q, m.w, m.vol, cfl=0.5)
    dtl = p64.compute_local_dt(0.5, pk.OWNER)
    p64.ctx.sync()
    assert report("E local dt", normwise(p64.nodes_out(dtl[None]), ref[None]), 1e-12)
    assert float(dtl.min()) == pytest.approx(oracle.dt(m.e2n, q, m.w, m.vol), rel=1e-12)


def test_gradient_and_second_order_full(prob_e, mesh_e):
    p64, _ = prob_e
    m, q = mesh_e
    dx = meshgen.edge_vectors(m)
    print("[E: oracle gradient and second-order residual]", flush=True)
    G_ref = oracle.gradient(m.e2n, q, m.w)
    r2_ref = oracle.residual2(m.e2n, q, G_ref, m.vol, m.w, dx)
    p64.set_edge_vectors(dx)
    G = torch.empty((18, m.N), dtype=torch.float64, device=DEV)
    p64.gradient(p64.qa, G, pk.OWNER, pk.WRITE)
    res = torch.empty((6, m.N), dtype=torch.float64, device=DEV)
    p64.residual2(p64.qa, G, res, pk.OWNER, pk.WRITE)
    p64.ctx.sync()
    assert report("E G", normwise(p64.nodes_out(G), G_ref), 1e-12)
    assert report("E res2", normwise(p64.nodes_out(res), r2_ref), 1e-12)


def test_geometry_full(mesh_e):
    m, q = mesh_e
    print("[E: tets and oracle geometry]", flush=True)
    t2n = m.tets()
    t2e = meshgen.tet_edges(m, t2n)
    w_ref, vol_ref = oracle.geometry(m.e2n, t2n, t2e, m.xyz)
    ctx = pk.Context(DEV)
    p = pk.FluxProblem(ctx, m.e2n, m.w, m.vol, q, coords=m.xyz, tets=t2n, tet_edges=t2e, **BENCH)
    x = p.nodes_in(m.xyz)
    rng = np.random.default_rng(42)
    wbar = rng.normal(size=(3, m.E))
    xb_ref = oracle.geometry_adjoint(m.e2n, t2n, t2e, m.xyz, wbar, np.zeros(m.N))
    wbar_d = p.nodes_in(wbar, edges=True)
    for variant in (pk.OWNER, pk.ATOMIC):
        # the gather form overwrites (WRITE); the scatter form adds into zeros
        fill = 1e30 if variant == pk.OWNER else 0.0
        w = torch.full((3, m.E), fill, dtype=torch.float64, device=DEV)
        vol = torch.full((m.N,), fill, dtype=torch.float64, device=DEV)
        p.geometry(x, w, vol, variant=variant, access=pk.WRITE if variant == pk.OWNER else pk.INC)
        p.ctx.sync()
        assert report(f"E geometry w v{variant}", normwise(p.nodes_out(w, edges=True), w_ref),
                      1e-12)
        assert report(f"E geometry vol v{variant}",
                      normwise(p.nodes_out(vol[None]), vol_ref[None]), 1e-12)
        del w, vol
        xbar = torch.zeros((3, m.N), dtype=torch.float64, device=DEV)
        p.geometry_adjoint(x, wbar_d, torch.zeros(m.N, dtype=torch.float64, device=DEV), xbar,
                           variant=variant)
        p.ctx.sync()
        assert report(f"E geometry xbar v{variant}", normwise(p.nodes_out(xbar), xb_ref), 1e-12)


def test_adjoint_sampled_full(prob_e, mesh_e):
    """qbar at sampled nodes and nbar at sampled edges, each formed one by one
    from the oracle's exact edge Jacobians."""
    p64, _ = prob_e
    m, q = mesh_e
    rbar = meshgen.normal(6 * m.N, purpose=21).reshape(6, m.N)
    rb = p64.nodes_in(rbar)
    qbar = torch.empty((6, m.N), dtype=torch.float64, device=DEV)
    nbar = torch.empty((3, m.E), dtype=torch.float64, device=DEV)
    p64.ctx.edge_flux_adjoint(p64.edges, p64.e2n, p64.dat(p64.qa), p64.w, p64.dat(rb),
                              p64.dat(qbar), p64.dat(nbar, edges=True), p64.gamma, pk.OWNER,
                              pk.WRITE)
    p64.ctx.sync()
    qbar_h = p64.nodes_out(qbar)
    nbar_h = p64.nodes_out(nbar, edges=True)
    rng = np.random.default_rng(64)
    nodes = rng.choice(m.N, 48, replace=False)
    inc = np.zeros(m.N, bool)
    inc[nodes] = True
    sel = np.nonzero(inc[m.e2n[:, 0]] | inc[m.e2n[:, 1]])[0]
    ref_q = {int(v): np.zeros(6) for v in nodes}
    for e in sel:
        i, j = m.e2n[e]
        _, J = oracle.edge_jacobian(q[:, i], q[:, j], m.w[:, e])
        Fb = rbar[:, i] - rbar[:, j]
        if inc[i]:
            ref_q[int(i)] += J[:, 0:6].T @ Fb
        if inc[j]:
            ref_q[int(j)] += J[:, 6:12].T @ Fb
    got = np.stack([qbar_h[:, v] for v in nodes], 1)
    ref = np.stack([ref_q[int(v)] for v in nodes], 1)
    assert report("E qbar (48 sampled nodes)", normwise(got, ref), 1e-12)
    edges = rng.choice(m.E, 64, replace=False)
    ref_n = []
    for e in edges:
        i, j = m.e2n[e]
        _, J = oracle.edge_jacobian(q[:, i], q[:, j], m.w[:, e])
        ref_n.append(J[:, 12:15].T @ (rbar[:, i] - rbar[:, j]))
    assert report("E nbar (64 sampled edges)", normwise(nbar_h[:, edges], np.stack(ref_n, 1)), 1e-12)


def test_fp32_trajectory_100_iterations():
    """The FP32-storage form over 100 iterations against the FP64 oracle
    trajectory on the 20^3 box (the oracle runs 500 residuals in seconds; the
    1M-node trajectory is in test_gpu_config_cd.py)."""
    m = meshgen.config_mesh("A")
    q = meshgen.state(m.N, m.perm)
    q32 = q.astype(np.float32).astype(np.float64)
    w32 = m.w.astype(np.float32).astype(np.float64)
    dt = oracle.dt(m.e2n, q32, w32, m.vol)
    ref = q32.copy()
    for _ in range(100):
        ref, _ = oracle.rk_iteration(m.e2n, ref, m.w, m.vol, dt)
    ctx = pk.Context(DEV)
    p32 = pk.FluxProblem(ctx, m.e2n, m.w, m.vol, q, fp32=True, coords=m.xyz, **BENCH)
    for _ in range(100):
        p32.rk_iteration(dt, pk.OWNER)
    ctx.sync()
    assert report("A fp32 100-iteration state", normwise(p32.nodes_out(p32.qa), ref), 1e-5)
    assert ctx.check_finite(p32.ss)


def test_adjoint_config_d():
    """The adjoint on the 1M-node jittered box: a dot-product test against the
    oracle's forward JVP on random directions (the whole-mesh comparison and the
    central differences are in test_gpu_config_cd.py)."""
    print("[1M-node jittered box: adjoint dot product]", flush=True)
    m = meshgen.config_mesh("D")
    q = meshgen.state(m.N, m.perm)
    ctx = pk.Context(DEV)
    p = pk.FluxProblem(ctx, m.e2n, m.w, m.vol, q, coords=m.xyz, **BENCH)
    rbar = meshgen.normal(6 * m.N, purpose=31).reshape(6, m.N)
    dq = meshgen.normal(6 * m.N, purpose=32).reshape(6, m.N) * np.abs(q).max(axis=1, keepdims=True)
    dw = meshgen.normal(3 * m.E, purpose=33).reshape(3, m.E) * np.abs(m.w).max()
    qbar = torch.empty((6, m.N), dtype=torch.float64, device=DEV)
    nbar = torch.empty((3, m.E), dtype=torch.float64, device=DEV)
    ctx.edge_flux_adjoint(p.edges, p.e2n, p.dat(p.qa), p.w, p.dat(p.nodes_in(rbar)), p.dat(qbar),
                          p.dat(nbar, edges=True), p.gamma, pk.OWNER, pk.WRITE)
    ctx.sync()
    qbar_h, nbar_h = p.nodes_out(qbar), p.nodes_out(nbar, edges=True)
    # <rbar, J (dq, dw)> = <qbar, dq> + <nbar, dw>
    jv = oracle.jvp(m.e2n, q, m.w, dq, dw)
    lhs = math.fsum((rbar * jv).ravel())
    rhs = math.fsum((qbar_h * dq).ravel()) + math.fsum((nbar_h * dw).ravel())
    rel = abs(lhs - rhs) / max(abs(lhs), abs(rhs))
    print(f"  dot product: {lhs:.15e} vs {rhs:.15e}, relative {rel:.3e}", flush=True)
    assert rel <= 1e-10
