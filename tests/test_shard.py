"""Owner-compute shards (host bookkeeping): the edges and halo one GPU of a
split mesh would hold, checked against the whole mesh."""
import numpy as np
import pytest

import meshgen
from paper_1403_7209_amd.shard import lattice_block, owner_shard


@pytest.fixture(scope="module")
def mesh():
    return meshgen.build_mesh(12, 1, 0.25)


def test_lattice_block_is_one_eighth(mesh):
    owned = lattice_block(mesh.xyz, 12, 3, 6)
    assert owned.sum() == 6 ** 3
    # the eight blocks of a 2x2x2 split cover every node once
    cover = np.zeros(mesh.N, dtype=np.int64)
    for a in (0, 6):
        for b in (0, 6):
            for c in (0, 6):
                idx = np.rint(mesh.xyz * 12).astype(np.int64) % 12
                blk = ((idx[0] >= a) & (idx[0] < a + 6) & (idx[1] >= b) & (idx[1] < b + 6)
                       & (idx[2] >= c) & (idx[2] < c + 6))
                cover += blk
    assert np.all(cover == 1)


def test_owner_shard_holds_every_edge_of_its_nodes(mesh):
    owned = lattice_block(mesh.xyz, 12, 3, 6)
    sh = owner_shard(mesh.e2n, owned)
    e2n = mesh.e2n.astype(np.int64)
    # exactly the edges with an owned end, in ascending order
    want = np.flatnonzero(owned[e2n[:, 0]] | owned[e2n[:, 1]])
    assert np.array_equal(sh.edges, want)
    # local endpoints map back to the global ones, orientation kept
    assert np.array_equal(sh.nodes[sh.e2n], e2n[sh.edges])
    # owned first, then halo, each ascending; halo = the other ends, none owned
    own = sh.nodes[:sh.n_owned]
    halo = sh.nodes[sh.n_owned:]
    assert np.array_equal(own, np.flatnonzero(owned))
    assert np.all(np.diff(own) > 0) and np.all(np.diff(halo) > 0)
    assert not owned[halo].any()
    assert np.array_equal(np.unique(sh.nodes[sh.e2n]), np.sort(sh.nodes))
    # every owned node keeps its whole star: the same degree as in the mesh
    deg = np.bincount(e2n.ravel(), minlength=mesh.N)
    deg_s = np.bincount(sh.e2n.ravel(), minlength=len(sh.nodes))
    assert np.array_equal(deg_s[:sh.n_owned], deg[own])
    # halo nodes keep only their edges into the owned block
    assert np.all(deg_s[sh.n_owned:] < deg[halo])
    # no edge joins two halo nodes
    assert np.all((sh.e2n[:, 0] < sh.n_owned) | (sh.e2n[:, 1] < sh.n_owned))


def test_owner_shards_of_a_split_cover_each_edge_once_or_twice(mesh):
    # every edge runs on the owner of each of its ends: once inside a block,
    # twice across a cut
    idx = np.rint(mesh.xyz * 12).astype(np.int64) % 12
    runs = np.zeros(mesh.E, dtype=np.int64)
    for a in (0, 6):
        for b in (0, 6):
            for c in (0, 6):
                owned = ((idx[0] >= a) & (idx[0] < a + 6) & (idx[1] >= b) & (idx[1] < b + 6)
                         & (idx[2] >= c) & (idx[2] < c + 6))
                runs[owner_shard(mesh.e2n, owned).edges] += 1
    blk = (idx[0] // 6) * 4 + (idx[1] // 6) * 2 + idx[2] // 6
    e2n = mesh.e2n.astype(np.int64)
    cut = blk[e2n[:, 0]] != blk[e2n[:, 1]]
    assert np.all(runs == np.where(cut, 2, 1))


def test_owner_shard_rejects_bad_input():
    with pytest.raises(ValueError):
        owner_shard(np.zeros((3, 3), np.int32), np.ones(4, bool))
    with pytest.raises(ValueError):
        owner_shard(np.array([[0, 5]], np.int32), np.ones(4, bool))


def test_owner_shard_degenerate_splits(mesh):
    # nothing owned: an empty share; everything owned: the whole mesh, no halo
    none = owner_shard(mesh.e2n, np.zeros(mesh.N, bool))
    assert none.n_owned == 0 and none.n_halo == 0 and len(none.edges) == 0
    assert none.e2n.shape == (0, 2)
    full = owner_shard(mesh.e2n, np.ones(mesh.N, bool))
    assert full.n_owned == mesh.N and full.n_halo == 0
    assert np.array_equal(full.edges, np.arange(mesh.E))
    assert np.array_equal(full.e2n, mesh.e2n)
    # one owned node: its star, with its neighbours as the halo
    one = np.zeros(mesh.N, bool)
    one[7] = True
    sh = owner_shard(mesh.e2n, one)
    e2n = mesh.e2n.astype(np.int64)
    star = np.flatnonzero((e2n[:, 0] == 7) | (e2n[:, 1] == 7))
    assert np.array_equal(sh.edges, star)
    assert sh.n_owned == 1 and sh.n_halo == len(star)
