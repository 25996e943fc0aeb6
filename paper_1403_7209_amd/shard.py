"""Owner-compute shards of an edge mesh: what one GPU of several would hold.

A GPU that owns a set of nodes runs every edge with at least one owned end
(an edge between two GPUs runs on both).  It reads the state of its halo, the
other ends of those edges, and its owned nodes' residuals are then complete
with no exchange of residuals; per stage it needs only the halo's new state.
This is the owner-compute rule of the distributed back-end (Sec. 3.2, halo
edges executed redundantly, Sec. 4.2), taken to GPUs; the library applies the
same rule to its workgroups.  Index bookkeeping on the host only: no part of
the method's arithmetic is here.
"""
from dataclasses import dataclass

import numpy as np


@dataclass
class Shard:
    nodes: np.ndarray   # (n_owned + n_halo,) global ids: owned ascending, then halo ascending
    edges: np.ndarray   # (E_s,) global ids of the edges with an owned end, ascending
    e2n: np.ndarray     # (E_s, 2) int32 endpoints in the shard's numbering (index into nodes)
    n_owned: int

    @property
    def n_halo(self):
        return len(self.nodes) - self.n_owned


def owner_shard(e2n, owned):
    """The shard of the nodes where `owned` (bool, (N,)) is set.  e2n: (E, 2)
    endpoints in global numbering.  Endpoint order within each edge is kept, so
    an edge's orientation (and the sign of its weight) is the same as in the
    whole mesh."""
    e2n = np.asarray(e2n)
    owned = np.asarray(owned, dtype=bool)
    if e2n.ndim != 2 or e2n.shape[1] != 2:
        raise ValueError("e2n must have shape (E, 2)")
    N = owned.shape[0]
    if e2n.size and (e2n.min() < 0 or e2n.max() >= N):
        raise ValueError("e2n refers to nodes outside the owned mask")
    keep = owned[e2n[:, 0]] | owned[e2n[:, 1]]
    edges = np.flatnonzero(keep)
    ends = e2n[edges]
    own_ids = np.flatnonzero(owned)
    touched = np.zeros(N, dtype=bool)
    touched[ends.ravel()] = True
    halo = np.flatnonzero(touched & ~owned)
    nodes = np.concatenate([own_ids, halo])
    local = np.full(N, -1, dtype=np.int64)
    local[nodes] = np.arange(len(nodes))
    return Shard(nodes=nodes, edges=edges, e2n=local[ends].astype(np.int32),
                 n_owned=int(len(own_ids)))


def lattice_block(xyz, n, lo, size):
    """Owned mask of the nodes of an n^3 lattice box (coordinates xyz (3, N) in
    [0, 1), each within half a spacing of its lattice point) whose lattice
    index lies in [lo, lo + size) along every axis: one block of a split of the
    box."""
    idx = np.rint(np.asarray(xyz) * n).astype(np.int64) % n
    return np.all((idx >= lo) & (idx < lo + size), axis=0)
