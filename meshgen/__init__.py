"""Seeded synthetic periodic tetrahedral meshes and node states.

The common input source of the oracle and the GPU path.  The meshes stand in
for the NASA Rotor 37 mesh of the paper's measurements (Sec. 4), which is not
available: node and edge sets, an arity-2 edge->node map, a 3-vector weight per
edge (three direct reads per edge, as in the edge loops of Table 2) and a
6-variable conservative state per node (at least six values per node, Sec. 3.1
and Sec. 4.1.2).  Nothing here evaluates the flux, the update or a reduction.
"""
import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

from . import _build

GAMMA = 1.4
MESH_SEED = 1403
STATE_SEED = 7209
DERIV_SEED = 2014

# Named workloads: n nodes per axis, split (0 Kuhn 6-tet, 1 layered 5/6 mix),
# jitter as a fraction of the lattice spacing.
CONFIGS = {
    "A": dict(n=20, split=0, jitter=0.0),
    "B": dict(n=100, split=0, jitter=0.2),
    "C": dict(n=100, split=0, jitter=0.2),
    "D": dict(n=100, split=0, jitter=0.2),
    "E": dict(n=160, split=1, jitter=0.25),
}


class _Params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("split", ctypes.c_int32),
                ("permute", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("jitter", ctypes.c_double), ("mesh_seed", ctypes.c_uint64)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        lib = ctypes.CDLL(_build.LIB)
        P = ctypes.POINTER
        i64p = P(ctypes.c_int64)
        lib.mg_sizes.argtypes = [P(_Params), i64p, i64p, i64p]
        lib.mg_build.argtypes = [P(_Params), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib.mg_tets.argtypes = [P(_Params), ctypes.c_void_p, ctypes.c_void_p]
        lib.mg_state.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_uint64,
                                 ctypes.c_double, ctypes.c_void_p]
        lib.mg_tet_dual.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib.mg_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_void_p]
        lib.mg_uniform.restype = None
        lib.mg_normal.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64,
                                  ctypes.c_void_p]
        lib.mg_normal.restype = None
        lib.mg_tet_edges.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                     ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Mesh:
    n: int
    split: int
    jitter: float
    seed: int
    N: int
    E: int
    T: int
    e2n: np.ndarray      # (E, 2) int32, user labels
    w: np.ndarray        # (3, E) float64 SoA edge weights, first -> second endpoint
    vol: np.ndarray      # (N,) float64 dual volumes
    xyz: np.ndarray      # (3, N) float64 positions
    perm: np.ndarray     # (N,) int32: user label of generator node g
    inverted: int = 0
    six_cubes: int = 0
    extra: dict = field(default_factory=dict)

    def tets(self):
        lib = _load()
        out = np.empty((self.T, 4), dtype=np.int32)
        p = _Params(self.n, self.split, 1, 0, self.jitter, self.seed)
        rc = lib.mg_tets(ctypes.byref(p), _ptr(self.perm), _ptr(out))
        if rc:
            raise RuntimeError(f"mg_tets failed ({rc})")
        return out


def edge_vectors(mesh):
    """(3, E) edge vectors x_j - x_i from the first to the second endpoint, taken
    across the periodic boundary where shorter (the unit box; jitter stays below
    a quarter of the spacing, so every edge is shorter than half the box)."""
    d = mesh.xyz[:, mesh.e2n[:, 1]] - mesh.xyz[:, mesh.e2n[:, 0]]
    return np.ascontiguousarray(d - np.round(d))


TET_LOCAL_EDGES = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))


def tet_edges(mesh, tets):
    """(T, 6) int32 edge ids of each tet's local edges in the order
    TET_LOCAL_EDGES (connectivity only: a lookup of node pairs in e2n)."""
    tets = np.ascontiguousarray(tets, dtype=np.int32)
    e2n = np.ascontiguousarray(mesh.e2n, dtype=np.int32)
    out = np.empty((tets.shape[0], 6), np.int32)
    rc = _load().mg_tet_edges(mesh.N, e2n.shape[0], _ptr(e2n), tets.shape[0], _ptr(tets),
                              _ptr(out))
    if rc == -1:
        raise ValueError("a tet edge is missing from the edge list")
    if rc:
        raise RuntimeError(f"mg_tet_edges failed ({rc})")
    return out


def smooth_state(mesh, amp=0.1, gamma=GAMMA):
    """A smooth periodic state: density 1 + amp sin(2 pi x) (x the first
    coordinate), uniform velocity (0.5, 0.2, -0.1), pressure 1, scalar 0.3."""
    rho = 1.0 + amp * np.sin(2 * np.pi * mesh.xyz[0])
    u = np.array([0.5, 0.2, -0.1])
    q = np.empty((6, mesh.N))
    q[0] = rho
    q[1:4] = rho[None, :] * u[:, None]
    q[4] = 1.0 / (gamma - 1.0) + 0.5 * rho * (u @ u)
    q[5] = 0.3 * rho
    return q


def sizes(n, split=0):
    lib = _load()
    p = _Params(n, split, 1, 0, 0.0, 0)
    N, E, T = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    if lib.mg_sizes(ctypes.byref(p), ctypes.byref(N), ctypes.byref(E), ctypes.byref(T)):
        raise ValueError(f"invalid mesh parameters n={n} split={split}")
    return N.value, E.value, T.value


def build_mesh(n, split=0, jitter=0.0, seed=MESH_SEED, permute=True):
    """Periodic tetrahedral mesh of the unit box with n^3 nodes."""
    lib = _load()
    N, E, T = sizes(n, split)
    p = _Params(n, split, 1 if permute else 0, 0, float(jitter), seed)
    e2n = np.empty((E, 2), dtype=np.int32)
    w = np.empty((3, E), dtype=np.float64)
    vol = np.empty(N, dtype=np.float64)
    xyz = np.empty((3, N), dtype=np.float64)
    perm = np.empty(N, dtype=np.int32)
    stats = np.zeros(3, dtype=np.int64)
    rc = lib.mg_build(ctypes.byref(p), _ptr(e2n), _ptr(w), _ptr(vol), _ptr(xyz), _ptr(perm),
                      _ptr(stats))
    if rc:
        raise RuntimeError(f"mg_build failed ({rc})")
    return Mesh(n, split, float(jitter), seed, N, E, T, e2n, w, vol, xyz, perm,
                int(stats[0]), int(stats[1]))


def config_mesh(name, seed=MESH_SEED, permute=True):
    c = CONFIGS[name]
    return build_mesh(c["n"], c["split"], c["jitter"], seed=seed, permute=permute)


def state(N, perm=None, seed=STATE_SEED, gamma=GAMMA):
    """Initial conservative state (6, N): rho, rho u, rho v, rho w, rho E, rho phi."""
    lib = _load()
    q = np.empty((6, N), dtype=np.float64)
    pp = _ptr(np.ascontiguousarray(perm, dtype=np.int32)) if perm is not None else None
    rc = lib.mg_state(N, pp, seed, gamma, _ptr(q))
    if rc:
        raise RuntimeError(f"mg_state failed ({rc})")
    return q


def uniform(count, lo=0.0, hi=1.0, seed=DERIV_SEED, purpose=11):
    out = np.empty(count, dtype=np.float64)
    _load().mg_uniform(seed, purpose, count, lo, hi, _ptr(out))
    return out


def normal(count, seed=DERIV_SEED, purpose=12):
    out = np.empty(count, dtype=np.float64)
    _load().mg_normal(seed, purpose, count, _ptr(out))
    return out


def tet_dual(x):
    """Six median-dual edge weights (edges 01,02,03,12,13,23) and the signed volume."""
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(12)
    nv = np.empty(18, dtype=np.float64)
    v = ctypes.c_double()
    _load().mg_tet_dual(_ptr(x), _ptr(nv), ctypes.byref(v))
    return nv.reshape(6, 3), v.value
