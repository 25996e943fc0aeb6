"""The allocation-free fused edge loop + stage (opf_edge_flux_stage_noalloc)
against the entry point it mirrors (opf_edge_flux_stage) and the oracle.

Two calls of the allocation-free entry point in a row, the second on a smaller
mesh (fewer owner clusters: the partial sums the first call left in the static
scratch beyond the second plan's clusters must not be read)."""
import numpy as np
import pytest
import torch

import meshgen
import oracle
import paper_1403_7209_amd as pk

from _util import normwise, report

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


def _one_stage(ctx, m, q, fp32, K, alpha):
    """Runs one fused stage through both entry points on a fresh problem;
    returns (qout, ss) of each, host float64 in user numbering."""
    p = pk.FluxProblem(ctx, m.e2n, m.w, m.vol, q, fp32=fp32, renumber="morton", coords=m.xyz,
                       cluster_size=K)
    assert p.info["nclusters"] > 1
    qa = p.dat(p.qa, "qa")
    out = {}
    for noalloc in (False, True):
        dst_t = torch.full_like(p.qa, float("nan"))
        ss = torch.zeros(6, dtype=torch.float64, device=ctx.torch_device)
        dst = p.dat(dst_t, "dst_noalloc" if noalloc else "dst")
        call = ctx.edge_flux_stage_noalloc if noalloc else ctx.edge_flux_stage
        call(p.edges, p.e2n, qa, p.w, qa, p.vol, dst, alpha, ss, p.gamma)
        ctx.sync()
        out[noalloc] = (p.nodes_out(dst_t).astype(np.float64), ss.cpu().numpy().copy())
    return p, out


def test_noalloc_fused_stage_matches_entry_point():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    ctx = pk.Context("cuda:0")
    alpha = 0.05
    # 4096 nodes in 16 clusters, then 1728 nodes in 7 clusters
    cases = [(16, False), (16, True), (12, False)]
    for n, fp32 in cases:
        m = meshgen.build_mesh(n, 1, 0.25)
        q = meshgen.state(m.N, m.perm)
        print(f"  case n={n} fp32={fp32} N={m.N} E={m.E}", flush=True)
        p, out = _one_stage(ctx, m, q, fp32, 256, alpha)
        tol = TOL32 if fp32 else TOL64
        assert report(f"noalloc vs entry point q n={n} fp32={fp32}",
                      normwise(out[True][0], out[False][0]), tol)
        assert report(f"noalloc vs entry point ss n={n} fp32={fp32}",
                      normwise(out[True][1], out[False][1]), tol)
        # the oracle: one stage q0 - alpha res / vol and sum res^2
        qin = q.astype(np.float32).astype(np.float64) if fp32 else q
        win = m.w.astype(np.float32).astype(np.float64) if fp32 else m.w
        res = oracle.residual(m.e2n, qin, win)
        q1 = qin - alpha * res / m.vol[None, :]
        ss_ref = (res * res).sum(axis=1)
        assert report(f"noalloc vs oracle q n={n} fp32={fp32}", normwise(out[True][0], q1), tol)
        assert report(f"noalloc vs oracle ss n={n} fp32={fp32}", normwise(out[True][1], ss_ref), tol)
    ctx.close()


def test_noalloc_refuses_without_plan_and_bad_args():
    """Argument checks of the allocation-free entry point run before anything
    is launched (aliasing of qout with q)."""
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    ctx = pk.Context("cuda:0")
    m = meshgen.build_mesh(8, 1, 0.2)
    q = meshgen.state(m.N, m.perm)
    p = pk.FluxProblem(ctx, m.e2n, m.w, m.vol, q, renumber="morton", coords=m.xyz, cluster_size=128)
    qa = p.dat(p.qa, "qa")
    ss = torch.zeros(6, dtype=torch.float64, device=ctx.torch_device)
    with pytest.raises(pk.OpfError):
        ctx.edge_flux_stage_noalloc(p.edges, p.e2n, qa, p.w, qa, p.vol, qa, 0.1, ss, p.gamma)
    ctx.close()
