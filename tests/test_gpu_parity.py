"""GPU parity of the edge-flux path against the FP64 oracle, through the C ABI.

Tolerances (normwise per variable, max |y - y*| / max |y*|):
  FP64 residual, stage update, sum of squares, time step, adjoint: 1e-12
  FP32-storage form from identical (FP32-rounded) inputs: 1e-5
The coloured variant must also be bitwise reproducible run to run.
"""
import numpy as np
import pytest
import torch

import meshgen
import oracle
import paper_1403_7209_amd as pk
from tests._util import normwise, report
from tests.golden.load import flux_hand_cases

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL64, TOL32 = 1e-12, 1e-5


ALL_VARIANTS = (pk.COLOURED, pk.ATOMIC, pk.OWNER, pk.COLOURED_LDS_ATOMIC, pk.FLAT)


def problem(m, q, fp32=False, renumber="rcm", block_size=512, colour_sort=False,
            cluster_size=512, lane_groups=True, owner_compact=False, bank_spread=True,
            halo_order=True):
    ctx = pk.Context(DEV)
    coords = m.xyz if renumber == "morton" else None
    return pk.FluxProblem(ctx, m.e2n, m.w, m.vol, q, fp32=fp32, renumber=renumber,
                          block_size=block_size, colour_sort=colour_sort, coords=coords,
                          cluster_size=cluster_size, lane_groups=lane_groups,
                          owner_compact=owner_compact, bank_spread=bank_spread,
                          halo_order=halo_order)


def variants(p):
    coloured = (pk.COLOURED, pk.COLOURED_LDS_ATOMIC)
    return [v for v in ALL_VARIANTS
            if (v != pk.OWNER or p.info["owner_ok"]) and (v != pk.FLAT or p.info["flat_ok"])
            and (v not in coloured or p.info["coloured_ok"])]


def gpu_residual(p, variant):
    res = torch.zeros((6, p.N), dtype=torch.float64, device=DEV)
    p.residual(p.qa, res, variant)
    p.ctx.sync()
    return p.nodes_out(res)


@pytest.mark.parametrize("variant", ALL_VARIANTS,
                         ids=["coloured", "atomic", "owner", "ldsatomic", "flat"])
@pytest.mark.parametrize("case", flux_hand_cases(), ids=lambda c: c[0])
def test_two_node_hand_cases(case, variant):
    name, qi, qj, n, F = case
    print(f"[two-node {name}]", flush=True)
    ctx = pk.Context(DEV)
    p = pk.FluxProblem(ctx, np.array([[0, 1]], np.int32), n.reshape(3, 1), np.ones(2),
                       np.stack([qi, qj], 1), block_size=64, cluster_size=64)
    res = gpu_residual(p, variant)
    assert np.abs(res[:, 0] - F).max() <= 1e-14 * np.abs(F).max()
    assert np.array_equal(res[:, 1], -res[:, 0])


MESHES = {
    "kuhn3": dict(n=3, split=0, jitter=0.2),
    "mix4": dict(n=4, split=1, jitter=0.25),
    "mix8": dict(n=8, split=1, jitter=0.25),
    "A": meshgen.CONFIGS["A"],
}


@pytest.fixture(scope="module", params=list(MESHES))
def small(request):
    c = MESHES[request.param]
    m = meshgen.build_mesh(c["n"], c["split"], c["jitter"])
    q = meshgen.state(m.N, m.perm)
    res = oracle.residual(m.e2n, q, m.w)
    return request.param, m, q, res


@pytest.mark.parametrize("renumber,bs,csort,K,lg,compact,spread,halo", [
    ("rcm", 512, False, 512, True, True, True, True),
    ("rcm", 512, False, 512, True, False, True, True),
    ("rcm", 64, True, 64, True, True, True, True),
    ("morton", 2048, False, 1024, False, True, True, True),
    ("morton", 256, False, 0, False, True, True, True),
    ("morton", 512, False, 512, True, False, False, False),
    ("morton", 512, False, 384, False, False, True, False),
    ("none", 256, False, 128, True, True, True, True),
    ("none", 256, False, 64, True, False, True, True)])
def test_residual_small(small, renumber, bs, csort, K, lg, compact, spread, halo):
    name, m, q, ref = small
    print(f"[residual {name} {renumber} bs={bs} sort={csort} K={K} groups={lg} compact={compact} "
          f"spread={spread} halo={halo}]", flush=True)
    p = problem(m, q, renumber=renumber, block_size=bs, colour_sort=csort, cluster_size=K,
                lane_groups=lg, owner_compact=compact, bank_spread=spread, halo_order=halo)
    assert p.info["owner_ok"] == (K > 0)
    assert p.info["owner_compact"] == (K > 0)
    for variant in variants(p):
        res = gpu_residual(p, variant)
        assert report(f"variant {variant}", normwise(res, ref), TOL64)
    # OP_INC accumulates into what is already there
    for variant in variants(p):
        res = torch.zeros((6, p.N), dtype=torch.float64, device=DEV)
        p.residual(p.qa, res, variant)
        p.residual(p.qa, res, variant)
        p.ctx.sync()
        assert normwise(p.nodes_out(res), 2 * ref) <= TOL64
    if p.info["owner_ok"]:
        # WRITE overwrites whatever the residual held
        res = torch.full((6, p.N), 1e30, dtype=torch.float64, device=DEV)
        p.residual(p.qa, res, pk.OWNER, res_access=pk.WRITE)
        p.ctx.sync()
        assert report("owner WRITE", normwise(p.nodes_out(res), ref), TOL64)
    else:
        with pytest.raises(pk.OpfError):
            gpu_residual(p, pk.OWNER)
    # WRITE is refused where a node's total is not formed in one place
    with pytest.raises(pk.OpfError) as e:
        p.residual(p.qa, torch.zeros((6, p.N), dtype=torch.float64, device=DEV), pk.COLOURED,
                   res_access=pk.WRITE)
    assert e.value.status == pk.EACCESS


def test_coloured_is_bitwise_deterministic(small):
    name, m, q, _ = small
    p = problem(m, q)
    a = gpu_residual(p, pk.COLOURED)
    b = gpu_residual(p, pk.COLOURED)
    assert a.tobytes() == b.tobytes()


def test_rk_stage_and_norm(small):
    name, m, q, ref = small
    print(f"[rk stage {name}]", flush=True)
    p = problem(m, q)
    rng = np.random.default_rng(1)
    res_h = ref * (1.0 + 0.1 * rng.standard_normal(ref.shape))
    q0 = q + 0.01 * rng.standard_normal(q.shape)
    q_ref, ss_ref = oracle.rk_stage(q0, res_h.copy(), m.vol, 0.37)
    q0_t = p.nodes_in(q0)
    res_t = p.nodes_in(res_h)
    out_t = torch.empty_like(q0_t)
    ss = torch.zeros(6, dtype=torch.float64, device=DEV)
    p.ctx.rk_stage(p.nodes, p.dat(q0_t), p.dat(res_t), p.vol, p.dat(out_t), 0.37, ss)
    p.ctx.sync()
    assert report("q", normwise(p.nodes_out(out_t), q_ref), TOL64)
    assert np.abs(ss.cpu().numpy() - ss_ref).max() <= TOL64 * np.abs(ss_ref).max()
    assert torch.count_nonzero(res_t).item() == 0


def test_time_step(small):
    name, m, q, _ = small
    p = problem(m, q)
    dt_ref = oracle.dt(m.e2n, q, m.w, m.vol)
    for variant in variants(p):
        dt = p.compute_dt(0.5, variant)
        assert abs(dt - dt_ref) <= TOL64 * dt_ref


def test_rk_iteration(small):
    name, m, q, _ = small
    print(f"[rk iteration {name}]", flush=True)
    dt = oracle.dt(m.e2n, q, m.w, m.vol)
    q_ref = q.copy()
    ss_ref = []
    for _ in range(2):
        q_ref, s = oracle.rk_iteration(m.e2n, q_ref, m.w, m.vol, dt)
        ss_ref.append(s)
    for variant in ALL_VARIANTS:
        p = problem(m, q)
        for it in range(2):
            p.rk_iteration(dt, variant)
            p.ctx.sync()
            rms = p.rms()
            assert report(f"rms it{it} v{variant}", normwise(rms, np.sqrt(ss_ref[it] / m.N)), TOL64)
        assert report(f"q v{variant}", normwise(p.nodes_out(p.qa), q_ref), TOL64)


def test_local_time_steps(small):
    """Per-node steps (spectral-radius loop + LOCAL_DT) and one 5-stage
    iteration with them, every variant, against the oracle."""
    name, m, q, _ = small
    print(f"[local time steps {name}]", flush=True)
    dtl_ref = oracle.local_dt(m.e2n, q, m.w, m.vol, cfl=0.5)
    q_ref, ss_ref = oracle.rk_iteration_local(m.e2n, q, m.w, m.vol, dtl_ref)
    p = problem(m, q)
    for variant in variants(p):
        p = problem(m, q)
        dtl = p.compute_local_dt(0.5, variant)
        p.ctx.sync()
        assert report(f"local dt v{variant}", normwise(p.nodes_out(dtl[None]), dtl_ref[None]),
                      TOL64)
        p.rk_iteration_local(variant)
        p.ctx.sync()
        assert report(f"local-step rms v{variant}", normwise(p.rms(), np.sqrt(ss_ref / m.N)),
                      TOL64)
        assert report(f"local-step q v{variant}", normwise(p.nodes_out(p.qa), q_ref), TOL64)


def test_gradient_and_second_order_flux(small):
    """Green-Gauss sums and the reconstructed (second-order) residual, every
    variant, against the oracle; the residual from the GPU's own sums."""
    name, m, q, _ = small
    print(f"[gradient + second order {name}]", flush=True)
    dx = meshgen.edge_vectors(m)
    G_ref = oracle.gradient(m.e2n, q, m.w)
    r2_ref = oracle.residual2(m.e2n, q, G_ref, m.vol, m.w, dx)
    p = problem(m, q)
    p.set_edge_vectors(dx)
    for variant in variants(p):
        G = torch.zeros((18, p.N), dtype=torch.float64, device=DEV)
        p.gradient(p.qa, G, variant)
        res = torch.zeros((6, p.N), dtype=torch.float64, device=DEV)
        p.residual2(p.qa, G, res, variant)
        p.ctx.sync()
        assert report(f"G v{variant}", normwise(p.nodes_out(G), G_ref), TOL64)
        assert report(f"res2 v{variant}", normwise(p.nodes_out(res), r2_ref), TOL64)
    if p.info["owner_ok"]:
        G = torch.full((18, p.N), 3e30, dtype=torch.float64, device=DEV)
        p.gradient(p.qa, G, pk.OWNER, pk.WRITE)
        res = torch.full((6, p.N), -5e30, dtype=torch.float64, device=DEV)
        p.residual2(p.qa, G, res, pk.OWNER, pk.WRITE)
        p.ctx.sync()
        assert report("G owner WRITE", normwise(p.nodes_out(G), G_ref), TOL64)
        assert report("res2 owner WRITE", normwise(p.nodes_out(res), r2_ref), TOL64)
    # the owner gradient runs two workgroups per cluster (a half of the sums
    # each) over a grid rounded up to 8 clusters: cluster counts that are not a
    # multiple of 8, and run-time cluster sizes
    for K in (96, 200):
        pk_ = problem(m, q, cluster_size=K)
        G = torch.full((18, pk_.N), 3e30, dtype=torch.float64, device=DEV)
        pk_.gradient(pk_.qa, G, pk.OWNER, pk.WRITE)
        pk_.ctx.sync()
        assert report(f"G owner K={K} ({pk_.info['nclusters']} clusters)",
                      normwise(pk_.nodes_out(G), G_ref), TOL64)


def test_geometry_and_shape_gradient(small):
    """Median-dual weights and volumes from the tets, their reverse, and the
    shape-sensitivity chain through the flux adjoint, against the oracle."""
    name, m, q, _ = small
    print(f"[geometry {name}]", flush=True)
    t2n = m.tets()
    t2e = meshgen.tet_edges(m, t2n)
    w_ref, vol_ref = oracle.geometry(m.e2n, t2n, t2e, m.xyz)
    ctx = pk.Context(DEV)
    p = pk.FluxProblem(ctx, m.e2n, m.w, m.vol, q, renumber="morton", coords=m.xyz,
                       tets=t2n, tet_edges=t2e)
    x = p.nodes_in(m.xyz)
    rng = np.random.default_rng(41)
    wbar, volbar = rng.normal(size=(3, m.E)), rng.normal(size=m.N)
    xb_ref = oracle.geometry_adjoint(m.e2n, t2n, t2e, m.xyz, wbar, volbar)
    for variant in (pk.OWNER, pk.ATOMIC):
        # the loop increments: start from values of the result's size (the mesh's
        # own weights and volumes), so that taking them off again loses nothing
        w0, vol0 = p.nodes_in(m.w, edges=True), p.nodes_in(m.vol[None])[0].contiguous()
        w, vol = w0.clone(), vol0.clone()
        p.geometry(x, w, vol, variant=variant)
        p.ctx.sync()
        assert report(f"geometry w v{variant}", normwise(p.nodes_out(w - w0, edges=True), w_ref),
                      TOL64)
        assert report(f"geometry vol v{variant}",
                      normwise(p.nodes_out((vol - vol0)[None]), vol_ref[None]), TOL64)
        xbar = torch.zeros((3, m.N), dtype=torch.float64, device=DEV)
        p.geometry_adjoint(x, p.nodes_in(wbar, edges=True),
                           p.nodes_in(volbar[None])[0].contiguous(), xbar, variant=variant)
        p.ctx.sync()
        assert report(f"geometry xbar v{variant}", normwise(p.nodes_out(xbar), xb_ref), TOL64)
    # the gather form sums in a fixed order: repeated calls agree bit for bit;
    # with WRITE access it overwrites whatever the outputs held
    w1 = torch.zeros((3, m.E), dtype=torch.float64, device=DEV)
    w2 = torch.full((3, m.E), 7.0e30, dtype=torch.float64, device=DEV)
    v1 = torch.zeros(m.N, dtype=torch.float64, device=DEV)
    v2 = torch.full((m.N,), -3.0e30, dtype=torch.float64, device=DEV)
    p.geometry(x, w1, v1)
    p.geometry(x, w2, v2, access=pk.WRITE)
    p.ctx.sync()
    assert torch.equal(w1, w2) and torch.equal(v1, v2)
    with pytest.raises(pk.OpfError):
        p.geometry(x, w2, v2, variant=pk.ATOMIC, access=pk.WRITE)
    # shape sensitivities of rbar . R(q, w(x))
    rbar = rng.normal(size=(6, m.N))
    _, nbar = oracle.adjoint(m.e2n, q, m.w, rbar)
    xs_ref = oracle.geometry_adjoint(m.e2n, t2n, t2e, m.xyz, nbar, np.zeros(m.N))
    for variant in variants(p):
        xs = p.shape_gradient(x, p.nodes_in(rbar), variant=variant)
        p.ctx.sync()
        assert report(f"shape gradient v{variant}", normwise(p.nodes_out(xs), xs_ref), TOL64)


def test_fused_stage_matches_separate_loops(small):
    """The owner loop with the stage update fused in gives the state and norms
    of the separate edge loop + stage update (and both the oracle's)."""
    name, m, q, _ = small
    dt = oracle.dt(m.e2n, q, m.w, m.vol)
    q_ref, ss_ref = oracle.rk_iteration(m.e2n, q, m.w, m.vol, dt)
    # clusters of 512 nodes (one per thread of the workgroup; partials through the
    # LDS tree), of 1024 (two per thread, same tree) and of 256 (the wavefront
    # reduction)
    for fp32, K in ((False, 512), (True, 512), (False, 1024), (False, 256)):
        runs = {}
        for fused in (True, False):
            p = problem(m, q, fp32=fp32, cluster_size=K)
            p.rk_iteration(dt, pk.OWNER, fused=fused)
            p.ctx.sync()
            runs[fused] = (p.nodes_out(p.qa).astype(np.float64), p.rms())
        tol = 1e-5 if fp32 else 1e-13
        tag = f"fp32={fp32} K={K}"
        assert report(f"fused vs separate q {tag}", normwise(runs[True][0], runs[False][0]), tol)
        assert report(f"fused vs separate rms {tag}", normwise(runs[True][1], runs[False][1]), tol)
        if not fp32:
            assert report(f"fused q vs oracle {tag}", normwise(runs[True][0], q_ref), TOL64)
            assert report(f"fused rms vs oracle {tag}", normwise(runs[True][1], np.sqrt(ss_ref / m.N)),
                          TOL64)


def test_fp32_storage_stage(small):
    name, m, q, _ = small
    q32 = q.astype(np.float32).astype(np.float64)
    w32 = m.w.astype(np.float32).astype(np.float64)
    ref = oracle.residual(m.e2n, q32, w32)
    p = problem(m, q, fp32=True)
    for variant in variants(p):
        res = gpu_residual(p, variant)
        assert report(f"fp32 residual v{variant}", normwise(res, ref), TOL32)
    dt = oracle.dt(m.e2n, q32, w32, m.vol)
    q1_ref, ss_ref = oracle.rk_iteration(m.e2n, q32, w32, m.vol, dt)
    for variant in (pk.COLOURED, pk.OWNER):
        p = problem(m, q, fp32=True)
        p.rk_iteration(dt, variant)
        p.ctx.sync()
        assert report(f"fp32 state v{variant}", normwise(p.nodes_out(p.qa), q1_ref), TOL32)
        assert report(f"fp32 rms v{variant}", normwise(p.rms(), np.sqrt(ss_ref / m.N)), TOL32)


def test_adjoint(small):
    name, m, q, _ = small
    print(f"[adjoint {name}]", flush=True)
    rbar = meshgen.normal(6 * m.N, purpose=21).reshape(6, m.N)
    qbar_ref, wbar_ref = oracle.adjoint(m.e2n, q, m.w, rbar)
    p = problem(m, q)
    rb = p.nodes_in(rbar)
    for variant in variants(p):
        qbar = torch.zeros((6, p.N), dtype=torch.float64, device=DEV)
        nbar = torch.empty((3, p.E), dtype=torch.float64, device=DEV)
        p.ctx.edge_flux_adjoint(p.edges, p.e2n, p.dat(p.qa), p.w, p.dat(rb), p.dat(qbar),
                                p.dat(nbar, edges=True), p.gamma, variant)
        p.ctx.sync()
        assert report(f"qbar v{variant}", normwise(p.nodes_out(qbar), qbar_ref), TOL64)
        assert report(f"nbar v{variant}", normwise(p.nodes_out(nbar, edges=True), wbar_ref), TOL64)
    if p.info["owner_ok"]:
        qbar = torch.full((6, p.N), -7.0, dtype=torch.float64, device=DEV)
        nbar = torch.full((3, p.E), -7.0, dtype=torch.float64, device=DEV)
        p.ctx.edge_flux_adjoint(p.edges, p.e2n, p.dat(p.qa), p.w, p.dat(rb), p.dat(qbar),
                                p.dat(nbar, edges=True), p.gamma, pk.OWNER, pk.WRITE)
        p.ctx.sync()
        assert report("qbar owner WRITE", normwise(p.nodes_out(qbar), qbar_ref), TOL64)
        assert normwise(p.nodes_out(nbar, edges=True), wbar_ref) <= TOL64


def test_autograd_dot_product_and_gradcheck():
    m = meshgen.build_mesh(3, 0, 0.2)
    q = meshgen.state(m.N, m.perm)
    p = problem(m, q)
    qt = p.qa.clone().requires_grad_(True)
    wt = p.w_t.clone().requires_grad_(True)
    res = pk.EdgeFluxFunction.apply(p, qt, wt, pk.COLOURED)
    rbar = torch.randn_like(res)
    qbar, wbar = torch.autograd.grad(res, (qt, wt), rbar)
    dq = torch.randn_like(qt)
    dw = torch.randn_like(wt) * wt.detach().norm(dim=0)
    jv = oracle.jvp(m.e2n, q, m.w, p.nodes_out(dq), p.nodes_out(dw, edges=True))
    lhs = float((p.nodes_out(rbar) * jv).sum())
    rhs = float((qbar * dq).sum() + (wbar * dw).sum())
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)
    f = lambda a, b: pk.EdgeFluxFunction.apply(p, a, b, pk.COLOURED)
    assert torch.autograd.gradcheck(f, (qt, wt), eps=1e-6, atol=1e-8, rtol=1e-6)


def test_argument_checks_on_device():
    m = meshgen.build_mesh(3, 0, 0.0)
    q = meshgen.state(m.N, m.perm)
    p = problem(m, q)
    res32 = torch.zeros((6, p.N), dtype=torch.float32, device=DEV)
    with pytest.raises(pk.OpfError) as e:
        p.ctx.edge_flux(p.edges, p.e2n, p.dat(p.qa), p.w, p.dat(res32), 1.4)
    assert e.value.status == pk.ETYPE
    short = torch.zeros((6, p.N), dtype=torch.float64, device=DEV)
    with pytest.raises(pk.OpfError) as e:  # a node dat passed where the edge weight goes
        p.ctx.edge_flux(p.edges, p.e2n, p.dat(p.qa), p.dat(short), p.dat(short), 1.4)
    assert e.value.status in (pk.EINVAL, pk.ESIZE)
    ss = torch.zeros(6, dtype=torch.float64, device=DEV)
    with pytest.raises(pk.OpfError) as e:  # q must not alias q0
        p.ctx.rk_stage(p.nodes, p.dat(p.qa), p.res_d, p.vol, p.dat(p.qa), 0.1, ss)
    assert e.value.status == pk.EINVAL
    with pytest.raises(pk.OpfError) as e:  # the stage never increments the residual
        p.ctx.rk_stage(p.nodes, p.dat(p.qa), p.res_d, p.vol, p.dat(p.qb), 0.1, ss,
                       res_access=pk.INC)
    assert e.value.status == pk.EACCESS
    # READ leaves the residual in place for a following WRITE edge loop
    res = torch.ones((6, p.N), dtype=torch.float64, device=DEV)
    p.ctx.rk_stage(p.nodes, p.dat(p.qa), p.dat(res), p.vol, p.dat(p.qb), 0.1, ss,
                   res_access=pk.READ)
    p.ctx.sync()
    assert bool((res == 1.0).all())
    nanq = p.qa.clone()
    nanq[0, 0] = float("nan")
    res = torch.zeros((6, p.N), dtype=torch.float64, device=DEV)
    p.residual(nanq, res)
    p.ctx.rk_stage(p.nodes, p.dat(p.qa), p.dat(res), p.vol, p.dat(p.qb), 0.1, ss)
    assert p.ctx.check_finite(ss) is False


def test_geometry_after_replanning():
    """A new plan renumbers the nodes and edges: the tet loops must follow it
    (their device copies of the tet maps are rebuilt, not reused).  1728 nodes:
    several chunks of the forward gather's ring form."""
    m = meshgen.build_mesh(12, 1, 0.25)
    t2n = m.tets()
    t2e = meshgen.tet_edges(m, t2n)
    w_ref, vol_ref = oracle.geometry(m.e2n, t2n, t2e, m.xyz)
    ctx = pk.Context(DEV)
    nodes = ctx.decl_set(m.N, "nodes")
    edges = ctx.decl_set(m.E, "edges")
    tets = ctx.decl_set(len(t2n), "tets")
    mp = ctx.decl_map(edges, nodes, 2, m.e2n, 0, "e2n")
    tn = ctx.decl_map(tets, nodes, 4, t2n, 0, "t2n")
    te = ctx.decl_map(tets, edges, 6, t2e, 0, "t2e")
    # the last plan has no owner clusters and colour-sorted partitions: its edges
    # are not grouped by chunks of nodes, and the forward gather uses per-tet records
    for renumber, K, cs in (("rcm", 128, False), ("morton", 128, False), ("none", 128, False),
                            ("morton", 0, True)):
        ctx.plan(mp, renumber=renumber, coords=m.xyz, block_size=256, cluster_size=K,
                 colour_sort=cs)
        node_new = ctx.get_perm(nodes, m.N)
        edge_new = ctx.get_perm(edges, m.E)
        x = np.empty((3, m.N))
        x[:, node_new] = m.xyz
        x_t = torch.from_numpy(x).to(DEV)
        for variant in (pk.OWNER, pk.ATOMIC):
            w = torch.zeros((3, m.E), dtype=torch.float64, device=DEV)
            vol = torch.zeros((1, m.N), dtype=torch.float64, device=DEV)
            ctx.geometry(tets, tn, te, ctx.decl_dat(nodes, x_t, "x"),
                         ctx.decl_dat(edges, w, "w"), ctx.decl_dat(nodes, vol, "vol"),
                         variant=variant)
            ctx.sync()
            tag = f"{renumber} K={K} v{variant}"
            assert report(f"geometry w after plan {tag}",
                          normwise(w.cpu().numpy()[:, edge_new], w_ref), TOL64)
            assert report(f"geometry vol after plan {tag}",
                          normwise(vol.cpu().numpy()[:, node_new], vol_ref[None]), TOL64)
    ctx.close()


def test_owner_and_atomic_without_colouring():
    """A map whose partitions cannot be coloured (a hub node in every
    partition): the plan keeps its owner clusters, the owner and atomic edge
    loops and the fused stage match the oracle, and the coloured variants
    refuse to run."""
    from tests.test_planner_abi import hub_map
    N, e2n = hub_map()
    print(f"[hub map: N={N} E={len(e2n)}]", flush=True)
    rng = np.random.default_rng(71)
    w = rng.normal(size=(3, len(e2n))) * 1e-2
    vol = np.full(N, 1e-3)
    q = meshgen.state(N)
    ctx = pk.Context(DEV)
    p = pk.FluxProblem(ctx, e2n, w, vol, q, renumber="none", cluster_size=512)
    assert p.info["coloured_ok"] == 0 and p.info["owner_ok"] == 1
    ref = oracle.residual(e2n, q, w)
    for variant in (pk.OWNER, pk.ATOMIC):
        assert report(f"hub residual v{variant}", normwise(gpu_residual(p, variant), ref), TOL64)
    for variant in (pk.COLOURED, pk.COLOURED_LDS_ATOMIC):
        with pytest.raises(pk.OpfError):
            gpu_residual(p, variant)
    dt = 1e-6  # the hub's 1100 edges: a small step keeps its state physical
    q1, ss = oracle.rk_iteration(e2n, q, w, vol, dt)
    p.rk_iteration(dt, pk.OWNER)
    ctx.sync()
    assert report("hub fused iteration", normwise(p.nodes_out(p.qa), q1), TOL64)
    ctx.close()


def test_geometry_bounded_mesh():
    """A mesh with a boundary (the tets of a periodic box that do not cross its
    seam, period 0): edges on the boundary have open fans of tets, whose chains
    do not close.  Both forms of the geometry loop and its reverse against the
    oracle, for chunks of 128 and 512 nodes."""
    m = meshgen.build_mesh(12, 1, 0.25)
    t_all = m.tets()
    x = m.xyz[:, t_all]  # (3, T, 4)
    keep = np.all(np.abs(x - x[:, :, :1]).max(axis=2) < 0.5, axis=0)
    t_old = t_all[keep]
    used = np.unique(t_old)
    new_id = np.full(m.N, -1, np.int64)
    new_id[used] = np.arange(len(used))
    t2n = new_id[t_old].astype(np.int32)
    xyz = np.ascontiguousarray(m.xyz[:, used])
    rng = np.random.default_rng(77)
    pairs = {tuple(sorted((int(a), int(b)))) for t in t2n
             for a, b in ((t[0], t[1]), (t[0], t[2]), (t[0], t[3]), (t[1], t[2]), (t[1], t[3]),
                          (t[2], t[3]))}
    e2n = np.array(sorted(pairs), dtype=np.int32)
    flip = rng.random(len(e2n)) < 0.5  # both orientations
    e2n[flip] = e2n[flip][:, ::-1]

    class _M:
        pass
    mm = _M()
    mm.N, mm.e2n = len(used), e2n
    t2e = meshgen.tet_edges(mm, t2n)
    N, E = len(used), len(e2n)
    print(f"[bounded mesh: {N} nodes, {E} edges, {len(t2n)} of {len(t_all)} tets]", flush=True)
    w_ref, vol_ref = oracle.geometry(e2n, t2n, t2e, xyz, period=0.0)
    wbar, volbar = rng.normal(size=(3, E)), rng.normal(size=N)
    xb_ref = oracle.geometry_adjoint(e2n, t2n, t2e, xyz, wbar, volbar, period=0.0)
    q = np.tile(np.array([1.0, 0.1, 0.0, 0.0, 2.5, 0.3])[:, None], (1, N))
    for K in (128, 512):
        ctx = pk.Context(DEV)
        p = pk.FluxProblem(ctx, e2n, np.zeros((3, E)), np.ones(N), q, renumber="morton",
                           coords=xyz, cluster_size=K, tets=t2n, tet_edges=t2e)
        xd = p.nodes_in(xyz)
        for variant in (pk.OWNER, pk.ATOMIC):
            w = torch.zeros((3, E), dtype=torch.float64, device=DEV)
            vol = torch.zeros(N, dtype=torch.float64, device=DEV)
            p.geometry(xd, w, vol, period=0.0, variant=variant)
            xbar = torch.zeros((3, N), dtype=torch.float64, device=DEV)
            p.geometry_adjoint(xd, p.nodes_in(wbar, edges=True),
                               p.nodes_in(volbar[None])[0].contiguous(), xbar, period=0.0,
                               variant=variant)
            p.ctx.sync()
            tag = f"K={K} v{variant}"
            assert report(f"bounded geometry w {tag}", normwise(p.nodes_out(w, edges=True), w_ref),
                          TOL64)
            assert report(f"bounded geometry vol {tag}",
                          normwise(p.nodes_out(vol[None]), vol_ref[None]), TOL64)
            assert report(f"bounded geometry xbar {tag}", normwise(p.nodes_out(xbar), xb_ref),
                          TOL64)
        ctx.close()
