"""One GPU's share of a mesh split over several (the owner-compute shard: the
owned nodes, their halo, every edge with an owned end) through the C ABI,
against the oracle run on the whole mesh: the owned nodes' residuals, states
after a fused stage and state adjoints, and the weight adjoints of every
shard edge, are those of the whole mesh.

Tolerances as in the parity tests: 1e-12 normwise FP64, 1e-5 for the
FP32-storage form from FP32-rounded inputs.
"""
import numpy as np
import pytest
import torch

import meshgen
import oracle
import paper_1403_7209_amd as pk
from paper_1403_7209_amd.shard import lattice_block, owner_shard
from tests._util import normwise, report

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL64, TOL32 = 1e-12, 1e-5
NB = 20  # nodes per axis; the shard is the central (NB/2)^3 block


@pytest.fixture(scope="module")
def case():
    m = meshgen.build_mesh(NB, 1, 0.25)
    q = meshgen.state(m.N, m.perm)
    sh = owner_shard(m.e2n, lattice_block(m.xyz, NB, NB // 4, NB // 2))
    print(f"[shard: {sh.n_owned} owned + {sh.n_halo} halo nodes, {len(sh.edges)} of {m.E} "
          f"edges]", flush=True)
    return m, q, sh


def shard_problem(m, q, sh, fp32=False, K=512):
    ctx = pk.Context(DEV)
    return pk.FluxProblem(ctx, sh.e2n, m.w[:, sh.edges], m.vol[sh.nodes], q[:, sh.nodes],
                          fp32=fp32, renumber="morton", coords=m.xyz[:, sh.nodes],
                          cluster_size=K)


@pytest.mark.parametrize("K", [512, 64])
def test_shard_residual(case, K):
    m, q, sh = case
    own = sh.nodes[:sh.n_owned]
    ref = oracle.residual(m.e2n, q, m.w)[:, own]
    p = shard_problem(m, q, sh, K=K)
    assert p.info["owner_ok"]
    for variant, acc in ((pk.OWNER, pk.WRITE), (pk.ATOMIC, pk.INC)):
        res = torch.zeros((6, p.N), dtype=torch.float64, device=DEV)
        p.residual(p.qa, res, variant, acc)
        p.ctx.sync()
        got = p.nodes_out(res)[:, :sh.n_owned]
        assert report(f"owned residual K={K} v{variant}", normwise(got, ref), TOL64)


def test_shard_fp32_residual(case):
    m, q, sh = case
    q32 = q.astype(np.float32).astype(np.float64)
    w32 = m.w.astype(np.float32).astype(np.float64)
    ref = oracle.residual(m.e2n, q32, w32)[:, sh.nodes[:sh.n_owned]]
    p = shard_problem(m, q, sh, fp32=True)
    res = torch.zeros((6, p.N), dtype=torch.float64, device=DEV)
    p.residual(p.qa, res, pk.OWNER, pk.WRITE)
    p.ctx.sync()
    assert report("owned FP32 residual", normwise(p.nodes_out(res)[:, :sh.n_owned], ref), TOL32)


def test_shard_fused_stage(case):
    m, q, sh = case
    own = sh.nodes[:sh.n_owned]
    adt = 0.37 * 1e-3
    q_ref, _ = oracle.rk_stage(q, oracle.residual(m.e2n, q, m.w), m.vol, adt)
    p = shard_problem(m, q, sh)
    out = torch.empty_like(p.qa)
    ss = torch.zeros(6, dtype=torch.float64, device=DEV)
    qa = p.dat(p.qa, "qa")
    p.ctx.edge_flux_stage(p.edges, p.e2n, qa, p.w, qa, p.vol, p.dat(out, "qb"), adt, ss,
                          p.gamma)
    p.ctx.sync()
    assert report("owned state after the fused stage",
                  normwise(p.nodes_out(out)[:, :sh.n_owned], q_ref[:, own]), TOL64)


def test_shard_adjoint(case):
    m, q, sh = case
    own = sh.nodes[:sh.n_owned]
    rbar = meshgen.normal(6 * m.N, purpose=21).reshape(6, m.N)
    qbar_ref, nbar_ref = oracle.adjoint(m.e2n, q, m.w, rbar)
    p = shard_problem(m, q, sh)
    rb = p.nodes_in(np.ascontiguousarray(rbar[:, sh.nodes]))
    qbar = torch.full((6, p.N), -7.0, dtype=torch.float64, device=DEV)
    nbar = torch.full((3, p.E), -7.0, dtype=torch.float64, device=DEV)
    p.ctx.edge_flux_adjoint(p.edges, p.e2n, p.dat(p.qa), p.w, p.dat(rb), p.dat(qbar),
                            p.dat(nbar, edges=True), p.gamma, pk.OWNER, pk.WRITE)
    p.ctx.sync()
    assert report("owned qbar", normwise(p.nodes_out(qbar)[:, :sh.n_owned], qbar_ref[:, own]),
                  TOL64)
    # every shard edge has an owned end, and both ends' states and seeds are there
    assert report("shard nbar", normwise(p.nodes_out(nbar, edges=True), nbar_ref[:, sh.edges]),
                  TOL64)


def test_whole_mesh_and_shard_on_one_context(case):
    # two problems on one context keep their own maps and plans
    m, q, sh = case
    ctx = pk.Context(DEV)
    whole = pk.FluxProblem(ctx, m.e2n, m.w, m.vol, q, renumber="morton", coords=m.xyz)
    part = pk.FluxProblem(ctx, sh.e2n, m.w[:, sh.edges], m.vol[sh.nodes], q[:, sh.nodes],
                          renumber="morton", coords=m.xyz[:, sh.nodes])
    ref = oracle.residual(m.e2n, q, m.w)
    for p, want, n in ((whole, ref, m.N), (part, ref[:, sh.nodes[:sh.n_owned]], sh.n_owned)):
        res = torch.empty((6, p.N), dtype=torch.float64, device=DEV)
        p.residual(p.qa, res, pk.OWNER, pk.WRITE)
        ctx.sync()
        assert report(f"residual, problem of {p.N} nodes", normwise(p.nodes_out(res)[:, :n], want),
                      TOL64)
