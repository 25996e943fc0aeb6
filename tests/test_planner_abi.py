"""Host-side tests of the C ABI: exports, declarations, the planner's integer
properties (checked here independently of the library's own verifier) and
the error paths that need no GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import meshgen
import paper_1403_7209_amd as pk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    with open(os.path.join(ROOT, "include", "opflux.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"^(?:int|const char \*)\s*(opf_\w+)\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(pk.LIB_PATH)
    names = declared_symbols()
    assert len(names) >= 19
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(pk.SYMBOLS)


def host_problem(m, **kw):
    ctx = pk.Context(None)
    nodes = ctx.decl_set(m.N, "nodes")
    edges = ctx.decl_set(m.E, "edges")
    mp = ctx.decl_map(edges, nodes, 2, m.e2n, 0, "e2n")
    info = ctx.plan(mp, coords=m.xyz, **kw)
    return ctx, nodes, edges, mp, info


def check_plan_properties(m, ctx, nodes, edges, mp):
    """Independent numpy check of the plan's properties 1-8."""
    v = ctx.plan_view(mp)
    node_new = ctx.get_perm(nodes, m.N)
    edge_new = ctx.get_perm(edges, m.E)
    # 1, 2: bijections; the internal map is the relabelled user map, orientation kept
    assert np.array_equal(np.sort(node_new), np.arange(m.N))
    assert np.array_equal(np.sort(edge_new), np.arange(m.E))
    e2n = v["e2n"]
    assert np.array_equal(e2n[edge_new], node_new[m.e2n])
    # 5: partitions are contiguous edge ranges of at most block_size edges
    off = v["block_offsets"]
    assert off[0] == 0 and off[-1] == m.E
    sizes = np.diff(off)
    assert sizes.min() >= 1 and sizes.max() <= v["block_size"]
    bcol = v["block_colour"]
    coff = v["colour_offsets"]
    assert np.array_equal(np.sort(v["colour_blocks"]), np.arange(v["nblocks"]))
    for c in range(v["nblock_colours"]):
        blocks = v["colour_blocks"][coff[c]:coff[c + 1]]
        assert len(blocks) > 0 and np.all(bcol[blocks] == c)
    blk_of_edge = np.repeat(np.arange(v["nblocks"]), sizes)
    # 6: local indices resolve to the map's nodes
    uoff = v["unique_offsets"]
    uniq = v["unique_nodes"]
    loc = v["local_idx"].astype(np.int64)
    for s in range(2):
        assert np.array_equal(uniq[uoff[blk_of_edge] + loc[:, s]], e2n[:, s])
    # 3: partitions of one colour share no node
    pair_col = np.repeat(bcol, np.diff(uoff))
    key = pair_col.astype(np.int64) * m.N + uniq
    assert len(np.unique(key)) == len(key)
    # 4: inside a partition, edges of one colour share no node
    ecol = v["elem_colour"].astype(np.int64)
    both = np.concatenate([e2n[:, 0], e2n[:, 1]]).astype(np.int64)
    k4 = (np.concatenate([blk_of_edge, blk_of_edge]) * 256 + np.concatenate([ecol, ecol])) * m.N + both
    assert len(np.unique(k4)) == len(k4)
    assert np.all(ecol < v["block_ncolours"][blk_of_edge])
    # 9: flat colouring: one colour per edge, no node twice in a colour
    nf = v["nflat_colours"]
    assert nf > 0
    fo, fe = v["flat_offsets"], v["flat_edges"]
    assert fo[0] == 0 and fo[-1] == m.E and np.all(np.diff(fo) > 0)
    assert np.array_equal(np.sort(fe), np.arange(m.E))
    fcol = np.repeat(np.arange(nf, dtype=np.int64), np.diff(fo))
    ends = e2n[fe].astype(np.int64)
    k9 = np.concatenate([fcol * m.N + ends[:, 0], fcol * m.N + ends[:, 1]])
    assert len(np.unique(k9)) == len(k9)
    # greedy colouring needs at most 2 * (max degree) - 1 colours
    deg = np.bincount(e2n.ravel(), minlength=m.N)
    assert nf <= 2 * deg.max() - 1
    # 8: every edge is run by exactly the owner clusters of its endpoints
    K = v["cluster_size"]
    if K:
        cnt = np.zeros(m.E, np.int64)
        soff = v["cluster_seg_offsets"]
        st, ln = v["cluster_seg_start"], v["cluster_seg_len"]
        for c in range(v["nclusters"]):
            for s in range(soff[c], soff[c + 1]):
                ks = np.arange(st[s], st[s] + ln[s])
                cl = e2n[ks] // K
                assert np.all((cl[:, 0] == c) | (cl[:, 1] == c))
                cnt[ks] += 1
        want = np.where(e2n[:, 0] // K == e2n[:, 1] // K, 1, 2)
        assert np.array_equal(cnt, want)
        # the visit lists hold the same work: the contiguous range of edges
        # whose smaller end the cluster owns (or nothing), then the rest
        cmin = e2n.min(axis=1) // K
        rng, loff, led = v["cluster_range"], v["cluster_list_offsets"], v["cluster_list_edges"]
        cnt[:] = 0
        contiguous = 0
        for c in range(v["nclusters"]):
            mine = np.nonzero(cmin == c)[0]
            r0, rn = rng[c]
            if rn:
                assert rn == len(mine) and r0 == mine[0] and mine[-1] == r0 + rn - 1
                contiguous += 1
            else:
                assert len(mine) == 0 or mine[-1] - mine[0] + 1 != len(mine)
            rest = led[loff[c]:loff[c + 1]]
            assert len(np.unique(rest)) == len(rest)
            ks = np.concatenate([np.arange(r0, r0 + rn), rest]).astype(np.int64)
            cl = e2n[ks] // K
            assert np.all((cl[:, 0] == c) | (cl[:, 1] == c))
            cnt[ks] += 1
        assert np.array_equal(cnt, want)
        # the owner kernel's two loops: the interior block (leading edges of the
        # range with both ends in the cluster), then one cut visit per other
        # (edge, owned end) pair; together every end of every edge exactly once
        ni, co = v["cluster_interior"], v["cluster_cut_offsets"]
        ce, ch = v["cluster_cut_edges"].astype(np.int64), v["cluster_cut_ends"].astype(np.int64)
        assert co[0] == 0 and co[-1] == len(ce) == len(ch) and np.all(np.diff(co) >= 0)
        assert np.all(ch <= 1)
        cover = np.zeros((m.E, 2), np.int64)
        for c in range(v["nclusters"]):
            r0, rn = rng[c]
            assert 0 <= ni[c] <= rn
            blk = np.arange(r0, r0 + ni[c])
            assert np.all(e2n[blk] // K == c)
            cover[blk] += 1
            es, hs = ce[co[c]:co[c + 1]], ch[co[c]:co[c + 1]]
            assert np.all(e2n[es, hs] // K == c)
            np.add.at(cover, (es, hs), 1)
            # the second order: the same (edge, end) pairs, sorted by foreign
            # node inside each run of one other cluster
            fs = v["cluster_cutf_edges"][co[c]:co[c + 1]].astype(np.int64)
            fh = v["cluster_cutf_ends"][co[c]:co[c + 1]].astype(np.int64)
            assert sorted(zip(es.tolist(), hs.tolist())) == sorted(zip(fs.tolist(), fh.tolist()))
            foreign = e2n[fs, 1 - fh]
            run = foreign // K
            starts = np.flatnonzero(np.r_[True, run[1:] != run[:-1]])
            for a, b in zip(starts, np.r_[starts[1:], len(run)]):
                assert np.all(np.diff(foreign[a:b]) >= 0)
        assert np.all(cover == 1)
        return contiguous / v["nclusters"]


@pytest.mark.parametrize("renumber,bs,K,lg,csort,spread,halo", [
    ("rcm", 512, 512, True, False, True, True),
    ("morton", 64, 64, True, True, True, True),
    ("none", 256, 0, False, False, True, True),
    ("morton", 2048, 4096, False, False, True, True),
    ("morton", 512, 128, True, False, False, True),
    ("rcm", 256, 256, False, False, True, False),
    ("morton", 512, 384, True, False, False, False)])
def test_plan_properties(renumber, bs, K, lg, csort, spread, halo):
    m = meshgen.build_mesh(8, 1, 0.25)
    ctx, nodes, edges, mp, info = host_problem(m, renumber=renumber, block_size=bs,
                                               cluster_size=K, lane_groups=lg,
                                               colour_sort=csort, bank_spread=spread,
                                               halo_order=halo)
    assert ctx.plan_verify(mp)["ok"]
    contiguous = check_plan_properties(m, ctx, nodes, edges, mp)
    assert info["nblocks"] == -(-m.E // bs)
    if K:
        assert info["owner_edge_visits"] >= m.E
        assert info["owner_ok"]
        # without the colour sort every cluster's own edges form one range
        assert csort or contiguous == 1.0


def hub_map(parts=1100, per=511):
    """A matching of 2 * per * parts nodes plus one hub node joined to one node
    of every run of `per` pairs: every partition holds a hub edge, so the
    partitions all conflict and need more colours than a plan allows."""
    M = 2 * per * parts
    pairs = np.stack([np.arange(0, M, 2), np.arange(1, M, 2)], 1)
    hub = np.stack([np.arange(0, M, 2 * per), np.full(parts, M)], 1)
    return M + 1, np.ascontiguousarray(np.concatenate([pairs, hub]).astype(np.int32))


def test_plan_degrades_per_variant():
    """When the two-level colouring cannot be built the plan stays valid for
    the owner clusters: coloured_ok is 0, the colouring arrays are absent, the
    owner kernel's work covers every edge end once, and the verifier passes."""
    N, e2n = hub_map()
    ctx = pk.Context(None)
    nodes = ctx.decl_set(N)
    edges = ctx.decl_set(len(e2n))
    mp = ctx.decl_map(edges, nodes, 2, e2n)
    info = ctx.plan(mp, renumber="none", cluster_size=512)
    assert info["coloured_ok"] == 0 and info["nblock_colours"] == 0
    assert info["owner_ok"] == 1
    assert ctx.plan_verify(mp)["ok"]
    v = ctx.plan_view(mp)
    assert v["block_colour"] is None and v["local_idx"] is None and v["unique_nodes"] is None
    K, ie = v["cluster_size"], v["e2n"].astype(np.int64)
    cover = np.zeros((len(e2n), 2), np.int64)
    rng, ni = v["cluster_range"], v["cluster_interior"]
    co, ce, ch = v["cluster_cut_offsets"], v["cluster_cut_edges"], v["cluster_cut_ends"]
    for c in range(v["nclusters"]):
        cover[rng[c, 0]:rng[c, 0] + ni[c]] += 1
        es, hs = ce[co[c]:co[c + 1]].astype(np.int64), ch[co[c]:co[c + 1]].astype(np.int64)
        assert np.all(ie[es, hs] // K == c)
        np.add.at(cover, (es, hs), 1)
    assert np.all(cover == 1)


def test_renumbering_reduces_bandwidth_and_verifier_on_config_a():
    m = meshgen.config_mesh("A")
    _, _, _, _, info = host_problem(m, renumber="rcm")
    assert info["bandwidth_after"] < info["bandwidth_before"] / 4
    ctx, nodes, edges, mp, info = host_problem(m, renumber="morton", block_size=256)
    check_plan_properties(m, ctx, nodes, edges, mp)
    # block colours per partition set are of the order the paper reports (tens)
    assert 2 <= info["nblock_colours"] <= 64


def test_lane_groups_make_wavefront_endpoints_distinct():
    m = meshgen.build_mesh(16, 1, 0.25)
    K = 512
    rates = {}
    for lg in (False, True):
        ctx, nodes, edges, mp, info = host_problem(m, renumber="morton", cluster_size=K,
                                                   lane_groups=lg)
        v = ctx.plan_view(mp)
        e2n = v["e2n"]
        rng, loff, led = v["cluster_range"], v["cluster_list_offsets"], v["cluster_list_edges"]
        rep = tot = 0
        for c in range(v["nclusters"]):
            # the order in which the owner kernel's lanes take the cluster's edges
            visits = np.concatenate([np.arange(rng[c, 0], rng[c, 0] + rng[c, 1]),
                                     led[loff[c]:loff[c + 1]]])
            for w0 in range(0, len(visits), 64):
                ends = e2n[visits[w0:w0 + 64]].ravel()
                own = ends[ends // K == c]
                tot += len(own)
                rep += len(own) - len(np.unique(own))
        rates[lg] = rep / tot
    assert rates[True] < 0.5 * rates[False]


def owner_bank_conflicts(v):
    """Excess same-bank LDS words over the owner kernel's wavefronts.  Interior
    loop: lanes run the cluster's interior block in order, each updating its
    edge's first and second end (the swap flag reverses them) with one LDS
    instruction each; cut loop: lanes run the cut visits in order, one owned end
    each.  The LDS serves a quarter-wave per pass with 16 banks of 8-byte words,
    so count equal offsets mod 16 per quarter-wave beyond the first."""
    K, e2n = v["cluster_size"], v["e2n"].astype(np.int64)
    rng, ni = v["cluster_range"], v["cluster_interior"]
    co, ce, ch = v["cluster_cut_offsets"], v["cluster_cut_edges"], v["cluster_cut_ends"]
    swap = v["owner_swap"]

    def excess(offsets):
        lane = np.arange(len(offsets)) % 64
        chunk = np.arange(len(offsets)) // 64
        key = (chunk * 4 + lane // 16) * 16 + offsets % 16
        _, cnt = np.unique(key, return_counts=True)
        return int((cnt - 1).sum())

    total = 0
    for c in range(v["nclusters"]):
        vis = np.arange(rng[c, 0], rng[c, 0] + ni[c])
        ends = e2n[vis].copy()
        if swap is not None:
            s = swap[vis].astype(bool)
            ends[s] = ends[s][:, ::-1]
        for slot in range(2):
            total += excess(ends[:, slot] - c * K)
        es, hs = ce[co[c]:co[c + 1]], ch[co[c]:co[c + 1]]
        total += excess(e2n[es, hs] - c * K)
    return total


def test_bank_spreading_cuts_lds_bank_conflicts():
    m = meshgen.build_mesh(16, 1, 0.25)
    out = {}
    for spread in (False, True):
        ctx, nodes, edges, mp, info = host_problem(m, renumber="morton", cluster_size=512,
                                                   bank_spread=spread)
        assert ctx.plan_verify(mp)["ok"]
        check_plan_properties(m, ctx, nodes, edges, mp)
        v = ctx.plan_view(mp)
        assert (v["owner_swap"] is not None) == spread
        out[spread] = owner_bank_conflicts(v)
    assert out[True] < 0.5 * out[False]


def halo_lines(m, node_new, K, L=16):
    """Distinct L-node lines of one state component that the clusters' foreign
    gathers touch, and the number of (cluster, foreign node) pairs."""
    a, b = node_new[m.e2n[:, 0]].astype(np.int64), node_new[m.e2n[:, 1]].astype(np.int64)
    cut = a // K != b // K
    g = np.concatenate([a[cut] // K, b[cut] // K])
    f = np.concatenate([b[cut], a[cut]])
    pairs = np.unique(g * m.N + f)
    return np.unique((pairs // m.N) * (m.N // L + 1) + (pairs % m.N) // L).size, pairs.size


def test_halo_order_groups_boundary_nodes():
    m = meshgen.build_mesh(24, 1, 0.25)
    K = 512
    lines = {}
    for ho in (False, True):
        ctx, nodes, edges, mp, info = host_problem(m, renumber="morton", cluster_size=K,
                                                   halo_order=ho)
        assert ctx.plan_verify(mp)["ok"]
        check_plan_properties(m, ctx, nodes, edges, mp)
        node_new = ctx.get_perm(nodes, m.N)
        lines[ho] = halo_lines(m, node_new, K)
        if not ho:
            base = node_new
            continue
        # the same clusters, only relabelled inside each one
        assert np.array_equal(base // K, node_new // K)
        # inside each cluster: interior nodes first, then boundary nodes in order of
        # (smallest, largest) other cluster they are joined to
        a, b = node_new[m.e2n[:, 0]], node_new[m.e2n[:, 1]]
        fmin = np.full(m.N, np.iinfo(np.int64).max)
        fmax = np.full(m.N, -1)
        cut = a // K != b // K
        for x, y in ((a, b), (b, a)):
            np.minimum.at(fmin, x[cut], y[cut] // K)
            np.maximum.at(fmax, x[cut], y[cut] // K)
        key = np.where(fmax < 0, -1, fmin) * (m.N // K + 2) + np.where(fmax < 0, -1, fmax)
        for c0 in range(0, m.N, K):
            k = key[c0:c0 + K]
            assert np.all(k[1:] >= k[:-1]), f"cluster at {c0} not grouped"
    assert lines[True][1] == lines[False][1]  # same halos
    assert lines[True][0] < 0.8 * lines[False][0]


def test_plan_is_deterministic():
    """The planner's parallel steps (bank spreading, halo order) split
    independent work only: planning the same map twice gives the same plan."""
    m = meshgen.build_mesh(16, 1, 0.25)
    views = []
    for _ in range(2):
        ctx, nodes, edges, mp, info = host_problem(m, renumber="morton", cluster_size=512)
        v = ctx.plan_view(mp)
        v["node_new"] = ctx.get_perm(nodes, m.N)
        v["edge_new"] = ctx.get_perm(edges, m.E)
        views.append(v)
    a, b = views
    for k, x in a.items():
        if isinstance(x, np.ndarray):
            assert np.array_equal(x, b[k]), k
        else:
            assert x == b[k], k


def test_declaration_errors():
    ctx = pk.Context(None)
    with pytest.raises(pk.OpfError) as e:
        ctx.decl_set(0)
    assert e.value.status == pk.ESIZE
    with pytest.raises(pk.OpfError) as e:
        ctx.decl_set(1 << 29)  # beyond 32-bit byte offsets of FP64 components
    assert e.value.status == pk.ESIZE
    nodes = ctx.decl_set(4, "nodes")
    edges = ctx.decl_set(3, "edges")
    with pytest.raises(pk.OpfError) as e:  # entry outside the target set
        ctx.decl_map(edges, nodes, 2, np.array([[0, 1], [1, 2], [2, 4]]), 0, "bad")
    assert e.value.status == pk.ERANGE
    # a 1-based map (as in the paper's Fortran declarations) is accepted with index_base 1
    mp = ctx.decl_map(edges, nodes, 2, np.array([[1, 2], [2, 3], [3, 4]]), 1, "e2n")
    ctx.plan(mp, block_size=64, cluster_size=64)
    v = ctx.plan_view(mp)
    node_new = ctx.get_perm(nodes, 4)
    edge_new = ctx.get_perm(edges, 3)
    assert np.array_equal(v["e2n"][edge_new], node_new[np.array([[0, 1], [1, 2], [2, 3]])])
    with pytest.raises(pk.OpfError) as e:
        ctx.decl_map(edges, nodes, 2, np.zeros((3, 2)), 2, "base2")
    assert e.value.status == pk.EINVAL


def test_plan_errors_and_stale_plans():
    ctx = pk.Context(None)
    nodes = ctx.decl_set(3, "nodes")
    edges = ctx.decl_set(2, "edges")
    loop = ctx.decl_map(edges, nodes, 2, np.array([[0, 1], [2, 2]]), 0, "loop")
    with pytest.raises(pk.OpfError) as e:  # an edge joining a node to itself
        ctx.plan(loop)
    assert e.value.status == pk.EINVAL
    ok = ctx.decl_map(edges, nodes, 2, np.array([[0, 1], [1, 2]]), 0, "loop")  # redeclared
    assert ok == loop
    with pytest.raises(pk.OpfError) as e:
        ctx.plan(ok, block_size=100)  # not a power of two
    assert e.value.status == pk.EINVAL
    with pytest.raises(pk.OpfError) as e:
        ctx.plan(ok, renumber="morton")  # Morton needs coordinates
    assert e.value.status == pk.EINVAL
    ctx.plan(ok, block_size=64, cluster_size=64)
    assert ctx.plan_verify(ok)["ok"]
    # re-declaring the map makes the plan stale: loops refuse it (host context:
    # the argument checks run before the device is touched)
    ctx.decl_map(edges, nodes, 2, np.array([[1, 0], [1, 2]]), 0, "loop")
    # a new map on sets a plan has renumbered would mix numberings: refused
    with pytest.raises(pk.OpfError) as e:
        ctx.decl_map(edges, nodes, 2, np.array([[0, 1], [1, 2]]), 0, "other")
    assert e.value.status == pk.ESTATE
    # a name already taken by a map between other sets, or of another arity, is
    # refused: the handle keeps its map
    cells = ctx.decl_set(2, "cells")
    with pytest.raises(pk.OpfError) as e:
        ctx.decl_map(cells, nodes, 2, np.array([[0, 1], [1, 2]]), 0, "loop")
    assert e.value.status == pk.EINVAL
    with pytest.raises(pk.OpfError) as e:
        ctx.decl_map(edges, nodes, 1, np.array([0, 1]), 0, "loop")
    assert e.value.status == pk.EINVAL
    assert ctx.decl_map(edges, nodes, 2, np.array([[1, 0], [1, 2]]), 0, "loop") == loop
    # plans are for arity-2 maps (the paper's cell->node example has arity 3)
    c2 = pk.Context(None)
    cells = c2.decl_set(2, "cells")
    verts = c2.decl_set(4, "nodes")
    tri = c2.decl_map(cells, verts, 3, np.array([[0, 1, 2], [1, 2, 3]]), 0, "pcell")
    with pytest.raises(pk.OpfError) as e:
        c2.plan(tri)
    assert e.value.status == pk.EINVAL


def test_loop_argument_checks_without_device():
    ctx = pk.Context(None)
    nodes = ctx.decl_set(3, "nodes")
    edges = ctx.decl_set(2, "edges")
    mp = ctx.decl_map(edges, nodes, 2, np.array([[0, 1], [1, 2]]), 0, "e2n")
    ctx.plan(mp, block_size=64, cluster_size=64)
    # host-only dats: NULL pointers are accepted on a host context
    lib = ctx.lib
    out = ctypes.c_int32()

    def dat(s, dim, typ, ld):
        assert lib.opf_decl_dat(ctx._ctx, s, dim, typ, None, ld, b"d", ctypes.byref(out)) == 0
        return out.value

    q = dat(nodes, 6, pk.F64, 3)
    n = dat(edges, 3, pk.F64, 2)
    res = dat(nodes, 6, pk.F64, 3)
    res32 = dat(nodes, 6, pk.F32, 3)
    assert lib.opf_decl_dat(ctx._ctx, nodes, 6, pk.F64, None, 2, b"short", ctypes.byref(out)) == pk.ESIZE
    assert lib.opf_decl_dat(ctx._ctx, nodes, 6, 7, None, 3, b"type", ctypes.byref(out)) == pk.ETYPE
    g = ctypes.c_double(1.4)

    def flux(args, gbl_dim=1, variant=pk.COLOURED):
        a = (pk.Arg * len(args))(*[pk.Arg(*x) for x in args])
        gb = (pk.Gbl * 1)(pk.Gbl(ctypes.addressof(g), gbl_dim, pk.F64, pk.READ, 0))
        return lib.opf_par_loop(ctx._ctx, pk.K_EDGE_FLUX, edges, len(args), a, 1, gb, variant, None)

    good = [(q, 0, mp, 6, pk.F64, pk.READ), (q, 1, mp, 6, pk.F64, pk.READ),
            (n, -1, pk.ID, 3, pk.F64, pk.READ), (res, 0, mp, 6, pk.F64, pk.INC),
            (res, 1, mp, 6, pk.F64, pk.INC)]
    assert flux(good) == pk.EDEVICE  # well-formed, but no device on this context
    bad_access = list(good)
    bad_access[3] = (res, 0, mp, 6, pk.F64, pk.READ)
    assert flux(bad_access) == pk.EACCESS
    bad_type = list(good)
    bad_type[3] = (res32, 0, mp, 6, pk.F32, pk.INC)
    bad_type[4] = (res32, 1, mp, 6, pk.F32, pk.INC)
    assert flux(bad_type) == pk.ETYPE
    bad_dim = list(good)
    bad_dim[2] = (n, -1, pk.ID, 2, pk.F64, pk.READ)
    assert flux(bad_dim) == pk.ESIZE
    bad_map = list(good)
    bad_map[2] = (n, 0, mp, 3, pk.F64, pk.READ)
    assert flux(bad_map) == pk.EINVAL
    assert flux(good[:4]) == pk.EINVAL
    assert flux(good, gbl_dim=2) == pk.ESIZE
    # WRITE increments only with the owner variant
    w = list(good)
    w[3] = (res, 0, mp, 6, pk.F64, pk.WRITE)
    w[4] = (res, 1, mp, 6, pk.F64, pk.WRITE)
    assert flux(w, variant=pk.COLOURED) == pk.EACCESS
    assert flux(w, variant=pk.OWNER) == pk.EDEVICE
    assert "host-only" in lib.opf_last_error(ctx._ctx).decode()
    assert flux(w, variant=pk.FLAT) == pk.EACCESS
    assert flux(good, variant=pk.FLAT) == pk.EDEVICE
    assert flux(good, variant=5) == pk.EINVAL
    # fused edge loop + stage: signature and aliasing
    q1 = dat(nodes, 6, pk.F64, 3)
    vol1s = dat(nodes, 1, pk.F64, 3)
    ssb = (ctypes.c_double * 6)()
    assert lib.opf_edge_flux_stage(ctx._ctx, edges, mp, q, n, q, vol1s, -1, q1, 1.4, 0.1,
                                   ctypes.addressof(ssb), None) == pk.EDEVICE
    assert lib.opf_edge_flux_stage(ctx._ctx, edges, mp, q, n, q, vol1s, -1, q, 1.4, 0.1,
                                   ctypes.addressof(ssb), None) == pk.EINVAL  # qout aliases q
    assert lib.opf_edge_flux_stage(ctx._ctx, edges, mp, q, n, q, q, -1, q1, 1.4, 0.1,
                                   ctypes.addressof(ssb), None) == pk.ESIZE  # vol of dim 6
    assert lib.opf_edge_flux_stage(ctx._ctx, edges, mp, q, n, q, vol1s, q1, q1, 1.4, 0.1,
                                   ctypes.addressof(ssb), None) == pk.ESIZE  # dt of dim 6
    # gradient and second-order loops: signatures
    G = dat(nodes, 18, pk.F64, 3)
    dx = dat(edges, 3, pk.F64, 2)
    assert lib.opf_edge_gradient(ctx._ctx, edges, mp, q, n, G, pk.COLOURED, pk.INC, None) == pk.EDEVICE
    assert lib.opf_edge_gradient(ctx._ctx, edges, mp, q, n, res, pk.COLOURED, pk.INC, None) == pk.ESIZE
    assert lib.opf_edge_gradient(ctx._ctx, edges, mp, q, n, G, pk.COLOURED, pk.WRITE, None) == pk.EACCESS
    assert lib.opf_edge_gradient(ctx._ctx, edges, mp, res32, n, G, pk.COLOURED, pk.INC, None) == pk.ETYPE
    vol1 = dat(nodes, 1, pk.F64, 3)
    assert lib.opf_edge_flux2(ctx._ctx, edges, mp, q, G, vol1, n, dx, res, 1.4, pk.OWNER, pk.WRITE,
                              None) == pk.EDEVICE
    assert lib.opf_edge_flux2(ctx._ctx, edges, mp, q, G, vol1, n, dx, q, 1.4, pk.COLOURED, pk.INC,
                              None) == pk.EINVAL  # increments into an input
    assert lib.opf_edge_flux2(ctx._ctx, edges, mp, q, res, vol1, n, dx, res, 1.4, pk.COLOURED,
                              pk.INC, None) == pk.ESIZE  # G of dimension 6
    assert lib.opf_edge_flux2(ctx._ctx, edges, mp, q, G, vol1, n, G, res, 1.4, pk.COLOURED, pk.INC,
                              None) == pk.EINVAL  # node dat where dx goes
    # local time steps: signatures of LOCAL_DT and of the stage with a step per node
    vol, lam, dtl = dat(nodes, 1, pk.F64, 3), dat(nodes, 1, pk.F64, 3), dat(nodes, 1, pk.F64, 3)
    edat = dat(edges, 1, pk.F64, 2)
    assert lib.opf_local_dt(ctx._ctx, nodes, vol, lam, 0.5, dtl, None) == pk.EDEVICE
    assert lib.opf_local_dt(ctx._ctx, nodes, vol, lam, 0.5, lam, None) == pk.EINVAL  # alias
    assert lib.opf_local_dt(ctx._ctx, nodes, vol, lam, 0.5, edat, None) == pk.EINVAL  # wrong set
    q0, q1 = dat(nodes, 6, pk.F64, 3), dat(nodes, 6, pk.F64, 3)
    assert lib.opf_rk_stage_local(ctx._ctx, nodes, q0, res, vol, dtl, q1, 0.25, None, pk.RW,
                                  None) == pk.EINVAL  # ss must be device memory
    ss = (ctypes.c_double * 6)()
    assert lib.opf_rk_stage_local(ctx._ctx, nodes, q0, res, vol, dtl, q1, 0.25,
                                  ctypes.addressof(ss), pk.RW, None) in (pk.EDEVICE, pk.EINVAL)
    assert lib.opf_rk_stage_local(ctx._ctx, nodes, q0, res, vol, q0, q1, 0.25,
                                  ctypes.addressof(ss), pk.RW, None) == pk.ESIZE  # dt of dim 6
    # a stale plan is refused
    ctx.decl_map(edges, nodes, 2, np.array([[0, 2], [1, 2]]), 0, "e2n")
    assert flux(good) == pk.ESTATE


def test_aliasing_is_checked_by_memory_without_device():
    """Outputs are compared with every other argument by the bytes they cover,
    not by handle: two handles declared over one buffer, or over overlapping
    parts of it, are refused before anything runs (host-only context, fake
    device addresses that are never dereferenced)."""
    m = meshgen.build_mesh(3, 0, 0.0)
    t2n = m.tets()
    t2e = meshgen.tet_edges(m, t2n)
    ctx = pk.Context(None)
    N, E, T = m.N, m.E, len(t2n)
    nodes, edges, tets = ctx.decl_set(N, "nodes"), ctx.decl_set(E, "edges"), ctx.decl_set(T, "tets")
    mp = ctx.decl_map(edges, nodes, 2, m.e2n, 0, "e2n")
    tn = ctx.decl_map(tets, nodes, 4, t2n, 0, "t2n")
    te = ctx.decl_map(tets, edges, 6, t2e, 0, "t2e")
    ctx.plan(mp, block_size=64, cluster_size=64)
    lib, out = ctx.lib, ctypes.c_int32()
    base = [1 << 40]

    def dat(s, dim, size, addr=None, typ=pk.F64):
        if addr is None:  # a fresh, disjoint fake region
            addr = base[0]
            base[0] += 1 << 24
        assert lib.opf_decl_dat(ctx._ctx, s, dim, typ, ctypes.c_void_p(addr), size, b"d",
                                ctypes.byref(out)) == 0
        return out.value, addr

    q, qa = dat(nodes, 6, N)
    n, na = dat(edges, 3, E)
    res, _ = dat(nodes, 6, N)
    res_on_q, _ = dat(nodes, 6, N, addr=qa)              # another handle, same memory
    res_tail_q, _ = dat(nodes, 6, N, addr=qa + 8 * (5 * N + N - 1))  # shares q's last value
    res_after_q, _ = dat(nodes, 6, N, addr=qa + 8 * 6 * N)  # starts right after q: disjoint
    V, C = pk.COLOURED, pk.OWNER
    assert lib.opf_edge_flux(ctx._ctx, edges, mp, q, n, res, 1.4, V, pk.INC, None) == pk.EDEVICE
    assert lib.opf_edge_flux(ctx._ctx, edges, mp, q, n, res_after_q, 1.4, V, pk.INC, None) == pk.EDEVICE
    for bad in (res_on_q, res_tail_q):
        assert lib.opf_edge_flux(ctx._ctx, edges, mp, q, n, bad, 1.4, V, pk.INC, None) == pk.EINVAL
        assert "overlaps" in lib.opf_last_error(ctx._ctx).decode()
    res_on_n, _ = dat(nodes, 6, N, addr=na)
    assert lib.opf_edge_flux(ctx._ctx, edges, mp, q, n, res_on_n, 1.4, C, pk.WRITE, None) == pk.EINVAL
    # adjoint: nbar must not share memory with n (nor with q, rbar or qbar)
    rbar, _ = dat(nodes, 6, N)
    qbar, qba = dat(nodes, 6, N)
    nbar, _ = dat(edges, 3, E)
    nbar_on_n, _ = dat(edges, 3, E, addr=na)
    nbar_on_qbar, _ = dat(edges, 3, E, addr=qba)
    adj = lib.opf_edge_flux_adjoint
    assert adj(ctx._ctx, edges, mp, q, n, rbar, qbar, nbar, 1.4, C, pk.WRITE, None) == pk.EDEVICE
    for bad in (nbar_on_n, nbar_on_qbar):
        assert adj(ctx._ctx, edges, mp, q, n, rbar, qbar, bad, 1.4, C, pk.WRITE, None) == pk.EINVAL
    # fused stage: qout against q0, vol and the device global ss
    q0, q0a = dat(nodes, 6, N)
    vol, vola = dat(nodes, 1, N)
    qout, _ = dat(nodes, 6, N)
    qout_on_q0, _ = dat(nodes, 6, N, addr=q0a)
    ssb = base[0]
    base[0] += 1 << 24
    fs = lib.opf_edge_flux_stage
    assert fs(ctx._ctx, edges, mp, q, n, q0, vol, -1, qout, 1.4, 0.1, ctypes.c_void_p(ssb),
              None) == pk.EDEVICE
    assert fs(ctx._ctx, edges, mp, q, n, q0, vol, -1, qout_on_q0, 1.4, 0.1, ctypes.c_void_p(ssb),
              None) == pk.EINVAL
    assert fs(ctx._ctx, edges, mp, q, n, q0, vol, -1, qout, 1.4, 0.1, ctypes.c_void_p(vola),
              None) == pk.EINVAL  # ss inside vol
    # RK stage: q against res; local dt: dt against vol
    q_on_res, _ = dat(nodes, 6, N, addr=base[0])
    res2, _ = dat(nodes, 6, N, addr=base[0])
    base[0] += 1 << 24
    assert lib.opf_rk_stage(ctx._ctx, nodes, q0, res2, vol, q_on_res, 0.1, ctypes.c_void_p(ssb),
                            pk.RW, None) == pk.EINVAL
    assert lib.opf_rk_stage(ctx._ctx, nodes, q0, res2, vol, qout, 0.1, ctypes.c_void_p(ssb),
                            pk.RW, None) == pk.EDEVICE
    lam, _ = dat(nodes, 1, N)
    dt_on_vol, _ = dat(nodes, 1, N, addr=vola)
    assert lib.opf_local_dt(ctx._ctx, nodes, vol, lam, 0.5, dt_on_vol, None) == pk.EINVAL
    # geometry: the volumes must not share memory with the coordinates
    x, xa = dat(nodes, 3, N)
    w, _ = dat(edges, 3, E)
    vol_on_x, _ = dat(nodes, 1, N, addr=xa + 8 * N)
    assert lib.opf_geometry(ctx._ctx, tets, tn, te, x, 1.0, w, vol, pk.OWNER, None) == pk.EDEVICE
    assert lib.opf_geometry(ctx._ctx, tets, tn, te, x, 1.0, w, vol_on_x, pk.OWNER, None) == pk.EINVAL


def test_tet_loop_checks_without_device():
    m = meshgen.build_mesh(4, 1, 0.25)
    t2n = m.tets()
    t2e = meshgen.tet_edges(m, t2n)
    ctx = pk.Context(None)
    nodes = ctx.decl_set(m.N, "nodes")
    edges = ctx.decl_set(m.E, "edges")
    tets = ctx.decl_set(len(t2n), "tets")
    mp = ctx.decl_map(edges, nodes, 2, m.e2n, 0, "e2n")
    tn = ctx.decl_map(tets, nodes, 4, t2n, 0, "t2n")
    te = ctx.decl_map(tets, edges, 6, t2e, 0, "t2e")
    lib, out = ctx.lib, ctypes.c_int32()

    def dat(s, dim):
        assert lib.opf_decl_dat(ctx._ctx, s, dim, pk.F64, None, ctx_size[s], b"d",
                                ctypes.byref(out)) == 0
        return out.value

    ctx_size = {nodes: m.N, edges: m.E, tets: len(t2n)}
    x, w, vol, xb = dat(nodes, 3), dat(edges, 3), dat(nodes, 1), dat(nodes, 3)
    O, A = pk.OWNER, pk.ATOMIC
    # before the plan the edges have no orientation map on the device
    assert lib.opf_geometry(ctx._ctx, tets, tn, te, x, 1.0, w, vol, O, None) == pk.ESTATE
    ctx.plan(mp, block_size=256, cluster_size=256)
    for v in (O, A):
        assert lib.opf_geometry(ctx._ctx, tets, tn, te, x, 1.0, w, vol, v, None) == pk.EDEVICE
    assert lib.opf_geometry(ctx._ctx, tets, tn, te, x, 1.0, w, vol, pk.FLAT, None) == pk.EINVAL
    assert lib.opf_geometry(ctx._ctx, tets, te, tn, x, 1.0, w, vol, O, None) == pk.EINVAL  # swapped
    assert lib.opf_geometry(ctx._ctx, tets, tn, te, x, -1.0, w, vol, O, None) == pk.EINVAL
    assert lib.opf_geometry(ctx._ctx, tets, tn, te, x, 1.0, w, x, O, None) == pk.ESIZE  # vol dim 3
    assert lib.opf_geometry_adjoint(ctx._ctx, tets, tn, te, x, 1.0, w, vol, xb, O,
                                    None) == pk.EDEVICE
    assert lib.opf_geometry_adjoint(ctx._ctx, tets, tn, te, x, 1.0, w, vol, x, O,
                                    None) == pk.EINVAL
    a = (pk.Arg * 3)(pk.Arg(x, pk.ALL, tn, 3, pk.F64, pk.READ), pk.Arg(w, pk.ALL, te, 3, pk.F64, pk.INC),
                     pk.Arg(vol, pk.ALL, tn, 1, pk.F64, pk.INC))
    period = ctypes.c_double(1.0)
    g = (pk.Gbl * 1)(pk.Gbl(ctypes.addressof(period), 1, pk.F64, pk.READ, 0))
    assert lib.opf_par_loop(ctx._ctx, pk.K_GEOMETRY, tets, 3, a, 1, g, pk.COLOURED, None) == pk.EINVAL
    assert lib.opf_par_loop(ctx._ctx, pk.K_GEOMETRY, tets, 3, a, 1, g, pk.ATOMIC, None) == pk.EDEVICE


def test_finalize_accepts_null_and_init_rejects_bad_device():
    lib = pk.load()
    assert lib.opf_finalize(None) == 0
    c = ctypes.c_void_p()
    assert lib.opf_init(ctypes.byref(c), -5) == pk.EINVAL
