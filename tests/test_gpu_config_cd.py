"""The FP64 loops (config B), the FP32-storage trajectory (config C) and the
adjoint (config D) on the 1M-node jittered box, against the FP64 oracle, in
the launch configuration bench.py times (owner variant, Morton renumbering,
clusters of 512 nodes).

B: the residual of every variant and one fused 5-stage iteration, bound at
1e-12 normwise.

C: 100 iterations of 5 stages with the stage update fused into the FP32
edge loop, each stage compared with the oracle's FP64 stage (the oracle fed
the unrounded FP64 inputs: the FP32 form's whole error), the state bound at
1e-5 normwise, the stage norms and residuals reported; and, for the first two
iterations, each stage from identical inputs (the oracle fed the GPU's FP32
state and FP32-rounded weights upcast to FP64), residual and norms bound at
1e-5.  The trajectory runs in five parts of 20 iterations sharing one state.

D: the adjoint's qbar and nbar over the whole mesh against the oracle's
dual-number adjoint; central differences of the local functionals on 64
seeded edges, bound per edge by 1e-6 times the largest adjoint value of the
edge's 15 inputs.
"""
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
ALPHA = pk.RK_ALPHA


@pytest.fixture(scope="module")
def traj_c():
    print("[config C: 1M-node jittered box, FP32 storage vs the FP64 oracle]", flush=True)
    m = meshgen.config_mesh("C")
    q = meshgen.state(m.N, m.perm)
    ctx = pk.Context(DEV)
    p = pk.FluxProblem(ctx, m.e2n, m.w, m.vol, q, fp32=True, coords=m.xyz, **BENCH)
    p.qc = torch.empty_like(p.qa)
    dt = oracle.dt(m.e2n, q, m.w, m.vol)
    w32 = m.w.astype(np.float32).astype(np.float64)
    state = dict(m=m, p=p, dt=dt, qref=q.copy(), w32=w32, it=0, worst_q=0.0, worst_rms=0.0,
                 worst_res=0.0)
    yield state
    print(f"  C over {state['it']} iterations: worst state error {state['worst_q']:.3e}, "
          f"worst stage rms error {state['worst_rms']:.3e} (reported)", flush=True)
    ctx.close()


def _advance(T, iters, identical_first=0):
    """Runs `iters` iterations on the GPU and in the oracle, stage by stage,
    comparing every stage; the first `identical_first` iterations also check
    each stage from identical inputs."""
    m, p, dt = T["m"], T["p"], T["dt"]
    N = m.N
    ss = torch.zeros((5, 6), dtype=torch.float64, device=DEV)
    res_gpu = torch.empty((6, N), dtype=torch.float64, device=DEV)
    for it in range(iters):
        qa = p.dat(p.qa, "qa")
        bufs = (p.dat(p.qb, "qb"), p.dat(p.qc, "qc"))
        tens = (p.qb, p.qc)
        src, src_t = qa, p.qa
        q0r, qkr = T["qref"], T["qref"]
        ss.zero_()
        errs_q, errs_rms = [], []
        for k in range(5):
            if it < identical_first:
                # (i) this stage from identical inputs: the GPU's FP32 state
                qin = p.nodes_out(src_t).astype(np.float64)
                r_same = oracle.residual(m.e2n, qin, T["w32"])
                p.residual(src_t, res_gpu, pk.OWNER, pk.WRITE)
                p.ctx.sync()
                e_res = normwise(p.nodes_out(res_gpu), r_same)
                assert report(f"C it {T['it']} stage {k}: residual, identical inputs", e_res, 1e-5)
            dst = bufs[k % 2]
            p.ctx.edge_flux_stage(p.edges, p.e2n, src, p.w, qa, p.vol, dst, ALPHA[k] * dt, ss[k],
                                  p.gamma)
            # the oracle's FP64 stage on the FP64 trajectory
            res = oracle.residual(m.e2n, qkr, m.w)
            if it < identical_first:
                q0in = p.nodes_out(p.qa).astype(np.float64)
                _, ss_same = oracle.rk_stage(q0in, r_same, m.vol, ALPHA[k] * dt)
            qkr, ss_ref = oracle.rk_stage(q0r, res, m.vol, ALPHA[k] * dt)
            p.ctx.sync()
            got = p.nodes_out(tens[k % 2]).astype(np.float64)
            eq = normwise(got, qkr)
            rms = np.sqrt(ss[k].cpu().numpy() / N)
            er = normwise(rms, np.sqrt(ss_ref / N))
            errs_q.append(eq)
            errs_rms.append(er)
            if it < identical_first:
                assert report(f"C it {T['it']} stage {k}: rms, identical inputs",
                              normwise(rms, np.sqrt(ss_same / N)), 1e-5)
            assert eq <= 1e-5, f"C iteration {T['it']} stage {k}: state error {eq:.3e}"
            src, src_t = dst, tens[k % 2]
        # stage 5 wrote qb: it becomes the next iteration's base state
        p.qa, p.qb = p.qb, p.qa
        T["qref"] = qkr
        T["worst_q"] = max(T["worst_q"], max(errs_q))
        T["worst_rms"] = max(T["worst_rms"], max(errs_rms))
        if T["it"] % 5 == 0 or it == iters - 1:
            print(f"  C it {T['it']}: state error per stage {['%.2e' % e for e in errs_q]}, "
                  f"rms error {['%.2e' % e for e in errs_rms]}", flush=True)
        T["it"] += 1


@pytest.mark.slow
@pytest.mark.parametrize("part", range(5))
def test_fp32_trajectory_vs_oracle_config_c(traj_c, part):
    assert traj_c["it"] == 20 * part, "the parts run in order on one trajectory"
    _advance(traj_c, 20, identical_first=2 if part == 0 else 0)
    assert torch.isfinite(traj_c["p"].qa).all()


def test_fp64_residual_and_iteration_config_b():
    """Config B (the same 1M-node box, FP64): the residual of every variant and
    one 5-stage iteration with the stage update fused into the owner loop,
    against the oracle."""
    print("[config B: 1M-node jittered box, FP64]", flush=True)
    m = meshgen.config_mesh("B")
    q = meshgen.state(m.N, m.perm)
    ctx = pk.Context(DEV)
    p = pk.FluxProblem(ctx, m.e2n, m.w, m.vol, q, coords=m.xyz, **BENCH)
    ref = oracle.residual(m.e2n, q, m.w)
    for variant in (pk.OWNER, pk.COLOURED, pk.COLOURED_LDS_ATOMIC, pk.ATOMIC, pk.FLAT):
        res = torch.zeros((6, m.N), dtype=torch.float64, device=DEV)
        p.residual(p.qa, res, variant)
        ctx.sync()
        assert report(f"B residual v{variant}", normwise(p.nodes_out(res), ref), 1e-12)
    dt = oracle.dt(m.e2n, q, m.w, m.vol)
    q1, ss = oracle.rk_iteration(m.e2n, q, m.w, m.vol, dt)
    p.rk_iteration(dt, pk.OWNER)
    ctx.sync()
    assert report("B fused iteration state", normwise(p.nodes_out(p.qa), q1), 1e-12)
    assert report("B fused iteration rms", normwise(p.rms(), np.sqrt(ss / m.N)), 1e-12)
    ctx.close()


@pytest.fixture(scope="module")
def adj_d():
    print("[config D: 1M-node jittered box, adjoint]", flush=True)
    m = meshgen.config_mesh("D")
    q = meshgen.state(m.N, m.perm)
    ctx = pk.Context(DEV)
    p = pk.FluxProblem(ctx, m.e2n, m.w, m.vol, q, coords=m.xyz, **BENCH)
    rbar = meshgen.normal(6 * m.N, purpose=31).reshape(6, m.N)
    qbar = torch.empty((6, m.N), dtype=torch.float64, device=DEV)
    nbar = torch.empty((3, m.E), dtype=torch.float64, device=DEV)
    ctx.edge_flux_adjoint(p.edges, p.e2n, p.dat(p.qa), p.w, p.dat(p.nodes_in(rbar)), p.dat(qbar),
                          p.dat(nbar, edges=True), p.gamma, pk.OWNER, pk.WRITE)
    ctx.sync()
    yield dict(m=m, q=q, p=p, rbar=rbar, qbar=p.nodes_out(qbar), nbar=p.nodes_out(nbar, edges=True))
    ctx.close()


def test_adjoint_whole_mesh_vs_oracle_config_d(adj_d):
    m, q, rbar = adj_d["m"], adj_d["q"], adj_d["rbar"]
    print("  oracle adjoint over 7M edges ...", flush=True)
    qb_ref, nb_ref = oracle.adjoint(m.e2n, q, m.w, rbar)
    assert report("D qbar, whole mesh", normwise(adj_d["qbar"], qb_ref), 1e-12)
    assert report("D nbar, whole mesh", normwise(adj_d["nbar"], nb_ref), 1e-12)


def test_adjoint_central_differences_config_d(adj_d):
    """For 64 seeded edges e = (i, j): the derivative of g_e = (rbar_i - rbar_j).F_e
    in n_e, and of G_i = sum over edges at i of (rbar_a - rbar_b).F in q_i (and
    G_j in q_j), by central differences of the GPU residual summed over the
    nodes the perturbation reaches, against nbar_e, qbar_i and qbar_j."""
    m, q, p, rbar = adj_d["m"], adj_d["q"], adj_d["p"], adj_d["rbar"]
    qbar, nbar = adj_d["qbar"], adj_d["nbar"]
    ends = np.concatenate([m.e2n[:, 0], m.e2n[:, 1]]).astype(np.int64)
    other = np.concatenate([m.e2n[:, 1], m.e2n[:, 0]]).astype(np.int64)
    order = np.argsort(ends, kind="stable")
    start = np.searchsorted(ends[order], np.arange(m.N + 1))

    def nbrs(v):
        return other[order[start[v]:start[v + 1]]].tolist()
    rb_d = torch.from_numpy(np.ascontiguousarray(rbar)).to(DEV)
    res = torch.empty((6, m.N), dtype=torch.float64, device=DEV)

    def functional(nodes_user):
        idx = torch.from_numpy(p.node_new[np.asarray(nodes_user)].astype(np.int64)).to(DEV)
        p.residual(p.qa, res, pk.OWNER, pk.WRITE)
        r = res[:, idx]
        rb = rb_d[:, torch.from_numpy(np.asarray(nodes_user, dtype=np.int64)).to(DEV)]
        return float((r * rb).sum())

    rng = np.random.default_rng(66)
    edges = rng.choice(m.E, 64, replace=False)
    worst = 0.0
    for e in edges:
        i, j = (int(x) for x in m.e2n[e])
        adj = np.concatenate([qbar[:, i], qbar[:, j], nbar[:, e]])
        fd = np.empty(15)
        ew = int(p.edge_new[e])
        for k in range(3):  # the weight vector: g_e, reached at i and j
            w0 = float(p.w_t[k, ew])
            h = 1e-6 * float(np.linalg.norm(m.w[:, e]))
            vals = []
            for s in (1.0, -1.0):
                p.w_t[k, ew] = w0 + s * h
                vals.append(functional([i, j]))
            p.w_t[k, ew] = w0
            fd[12 + k] = (vals[0] - vals[1]) / (2 * h)
        for slot, v in ((0, i), (1, j)):  # the state of an end: G_v, reached at v and its neighbours
            reach = [v] + nbrs(v)
            vi = int(p.node_new[v])
            for c in range(6):
                x0 = float(p.qa[c, vi])
                h = 1e-6 * max(1.0, abs(x0))
                vals = []
                for s in (1.0, -1.0):
                    p.qa[c, vi] = x0 + s * h
                    vals.append(functional(reach))
                p.qa[c, vi] = x0
                fd[6 * slot + c] = (vals[0] - vals[1]) / (2 * h)
        err = np.abs(adj - fd).max() / np.abs(adj).max()
        worst = max(worst, err)
        assert err <= 1e-6, f"edge {e}: central differences {err:.3e}"
    print(f"  D central differences on 64 edges (15 inputs each): worst {worst:.3e} "
          f"of the edge's largest adjoint value", flush=True)
