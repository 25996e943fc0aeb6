"""Sequential FP64 CPU oracle of the edge-flux hot path.

TEST INFRASTRUCTURE: only tests/, __graft_entry__.smoke() and the CPU baseline
leg of bench.py may import this package.  It never touches the GPU library.

Arrays follow the library's user-facing layout: q (6, N), w (3, E), vol (N,),
e2n (E, 2) int32, all host numpy arrays in user numbering.
"""
import ctypes
import os

import numpy as np

from . import _build

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        lib = ctypes.CDLL(_build.LIB)
        vp, i64, d = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double
        lib.orc_rk_alpha.argtypes = [ctypes.c_int]
        lib.orc_rk_alpha.restype = d
        lib.orc_flux.argtypes = [vp, vp, vp, d, vp]
        lib.orc_flux.restype = None
        lib.orc_residual.argtypes = [i64, i64, vp, vp, vp, d, vp, vp]
        lib.orc_rk_stage.argtypes = [i64, vp, vp, vp, d, vp, vp]
        lib.orc_rk_iteration.argtypes = [i64, i64, vp, vp, vp, vp, d, d, vp]
        lib.orc_spectral_radius.argtypes = [i64, i64, vp, vp, vp, d, vp]
        lib.orc_dt.argtypes = [i64, i64, vp, vp, vp, vp, d, d]
        lib.orc_local_dt.argtypes = [i64, i64, vp, vp, vp, vp, d, d, vp]
        lib.orc_rk_stage_local.argtypes = [i64, vp, vp, vp, vp, d, vp, vp]
        lib.orc_rk_iteration_local.argtypes = [i64, i64, vp, vp, vp, vp, d, vp, vp]
        lib.orc_dt.restype = d
        lib.orc_gradient.argtypes = [i64, i64, vp, vp, vp, vp]
        lib.orc_residual2.argtypes = [i64, i64, vp, vp, vp, vp, vp, vp, d, vp]
        lib.orc_geometry.argtypes = [i64, i64, i64, vp, vp, vp, vp, d, vp, vp]
        lib.orc_geometry_adjoint.argtypes = [i64, i64, i64, vp, vp, vp, vp, d, vp, vp, vp]
        lib.orc_jvp.argtypes = [i64, i64, vp, vp, vp, d, vp, vp, vp]
        lib.orc_edge_jacobian.argtypes = [vp, vp, vp, d, vp, vp]
        lib.orc_adjoint.argtypes = [i64, i64, vp, vp, vp, d, vp, vp, vp]
        _lib = lib
    return _lib


def _c(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(rc, what):
    if rc:
        raise RuntimeError(f"{what} failed with status {rc}")


RK_ALPHA = None


def rk_alpha():
    return [_load().orc_rk_alpha(k) for k in range(5)]


def flux(qi, qj, n, gamma=1.4):
    F = np.empty(6)
    _load().orc_flux(_p(_c(qi)), _p(_c(qj)), _p(_c(n)), gamma, _p(F))
    return F


def residual(e2n, q, w, gamma=1.4, res=None, with_scale=False):
    """res (6, N) += sum_e (+F at first node, -F at second); optionally |F| scale."""
    e2n = _c(e2n, np.int32)
    q, w = _c(q), _c(w)
    N, E = q.shape[1], w.shape[1]
    out = np.zeros((6, N)) if res is None else res
    S = np.zeros((6, N)) if with_scale else None
    _check(_load().orc_residual(N, E, _p(e2n), _p(q), _p(w), gamma, _p(out), _p(S)),
           "orc_residual")
    return (out, S) if with_scale else out


def rk_stage(q0, res, vol, alpha_dt):
    """Returns (q, ss[6]); res is zeroed in place."""
    q0, vol = _c(q0), _c(vol)
    assert res.flags.c_contiguous and res.dtype == np.float64
    N = q0.shape[1]
    q = np.empty_like(q0)
    ss = np.empty(6)
    _check(_load().orc_rk_stage(N, _p(q0), _p(res), _p(vol), alpha_dt, _p(q), _p(ss)),
           "orc_rk_stage")
    return q, ss


def rk_iteration(e2n, q0, w, vol, dt, gamma=1.4):
    """One 5-stage iteration; returns (q, ss (5, 6))."""
    e2n = _c(e2n, np.int32)
    q = _c(q0).copy()
    w, vol = _c(w), _c(vol)
    ss = np.empty(30)
    _check(_load().orc_rk_iteration(q.shape[1], w.shape[1], _p(e2n), _p(q), _p(w), _p(vol),
                                    gamma, dt, _p(ss)), "orc_rk_iteration")
    return q, ss.reshape(5, 6)


def spectral_radius(e2n, q, w, gamma=1.4):
    e2n, q, w = _c(e2n, np.int32), _c(q), _c(w)
    out = np.zeros(q.shape[1])
    _check(_load().orc_spectral_radius(q.shape[1], w.shape[1], _p(e2n), _p(q), _p(w), gamma,
                                       _p(out)), "orc_spectral_radius")
    return out


def dt(e2n, q, w, vol, gamma=1.4, cfl=0.5):
    e2n, q, w, vol = _c(e2n, np.int32), _c(q), _c(w), _c(vol)
    r = _load().orc_dt(q.shape[1], w.shape[1], _p(e2n), _p(q), _p(w), _p(vol), gamma, cfl)
    if r < 0:
        raise RuntimeError("orc_dt failed")
    return r


def local_dt(e2n, q, w, vol, gamma=1.4, cfl=0.5):
    """Per-node time step cfl * vol_i / sum of lambda_e at i."""
    e2n, q, w, vol = _c(e2n, np.int32), _c(q), _c(w), _c(vol)
    out = np.empty(q.shape[1])
    _check(_load().orc_local_dt(q.shape[1], w.shape[1], _p(e2n), _p(q), _p(w), _p(vol), gamma,
                                cfl, _p(out)), "orc_local_dt")
    return out


def rk_stage_local(q0, res, vol, dt, alpha):
    """Returns (q, ss[6]) with a time step per node; res is zeroed in place."""
    q0, vol, dt = _c(q0), _c(vol), _c(dt)
    assert res.flags.c_contiguous and res.dtype == np.float64
    q = np.empty_like(q0)
    ss = np.empty(6)
    _check(_load().orc_rk_stage_local(q0.shape[1], _p(q0), _p(res), _p(vol), _p(dt), alpha, _p(q),
                                      _p(ss)), "orc_rk_stage_local")
    return q, ss


def rk_iteration_local(e2n, q0, w, vol, dt, gamma=1.4):
    """One 5-stage iteration with per-node time steps dt; returns (q, ss (5, 6))."""
    e2n = _c(e2n, np.int32)
    q = _c(q0).copy()
    w, vol, dt = _c(w), _c(vol), _c(dt)
    ss = np.empty(30)
    _check(_load().orc_rk_iteration_local(q.shape[1], w.shape[1], _p(e2n), _p(q), _p(w), _p(vol),
                                          gamma, _p(dt), _p(ss)), "orc_rk_iteration_local")
    return q, ss.reshape(5, 6)


def gradient(e2n, q, w):
    """Green-Gauss sums G (18, N), component (v, d) in row 3v + d; gradient = G / vol."""
    e2n, q, w = _c(e2n, np.int32), _c(q), _c(w)
    G = np.zeros((18, q.shape[1]))
    _check(_load().orc_gradient(q.shape[1], w.shape[1], _p(e2n), _p(q), _p(w), _p(G)),
           "orc_gradient")
    return G


def residual2(e2n, q, G, vol, w, dx, gamma=1.4):
    """Second-order residual from Green-Gauss sums G (18, N) and edge vectors dx (3, E)."""
    e2n, q, G, vol, w, dx = (_c(e2n, np.int32), _c(q), _c(G), _c(vol), _c(w), _c(dx))
    res = np.zeros((6, q.shape[1]))
    _check(_load().orc_residual2(q.shape[1], w.shape[1], _p(e2n), _p(q), _p(G), _p(vol), _p(w),
                                 _p(dx), gamma, _p(res)), "orc_residual2")
    return res


def geometry(e2n, t2n, t2e, xyz, period=1.0):
    """Median-dual edge weights (3, E) and node volumes (N,) of the tets."""
    e2n, t2n, t2e, xyz = _c(e2n, np.int32), _c(t2n, np.int32), _c(t2e, np.int32), _c(xyz)
    N, E, T = xyz.shape[1], e2n.shape[0], t2n.shape[0]
    w, vol = np.zeros((3, E)), np.zeros(N)
    _check(_load().orc_geometry(N, E, T, _p(e2n), _p(t2n), _p(t2e), _p(xyz), period, _p(w),
                                _p(vol)), "orc_geometry")
    return w, vol


def geometry_adjoint(e2n, t2n, t2e, xyz, wbar, volbar, period=1.0):
    """xbar (3, N) = (dw/dx)^T wbar + (dvol/dx)^T volbar."""
    e2n, t2n, t2e, xyz = _c(e2n, np.int32), _c(t2n, np.int32), _c(t2e, np.int32), _c(xyz)
    wbar, volbar = _c(wbar), _c(volbar)
    N, E, T = xyz.shape[1], e2n.shape[0], t2n.shape[0]
    xbar = np.zeros((3, N))
    _check(_load().orc_geometry_adjoint(N, E, T, _p(e2n), _p(t2n), _p(t2e), _p(xyz), period,
                                        _p(wbar), _p(volbar), _p(xbar)), "orc_geometry_adjoint")
    return xbar


def jvp(e2n, q, w, dq=None, dw=None, gamma=1.4):
    e2n, q, w = _c(e2n, np.int32), _c(q), _c(w)
    dq = None if dq is None else _c(dq)
    dw = None if dw is None else _c(dw)
    jv = np.empty_like(q)
    _check(_load().orc_jvp(q.shape[1], w.shape[1], _p(e2n), _p(q), _p(w), gamma, _p(dq),
                           _p(dw), _p(jv)), "orc_jvp")
    return jv


def edge_jacobian(qi, qj, n, gamma=1.4):
    F = np.empty(6)
    J = np.empty((6, 15))
    _load().orc_edge_jacobian(_p(_c(qi)), _p(_c(qj)), _p(_c(n)), gamma, _p(F), _p(J))
    return F, J


def adjoint(e2n, q, w, rbar, gamma=1.4):
    """Returns (qbar (6, N), wbar (3, E))."""
    e2n, q, w, rbar = _c(e2n, np.int32), _c(q), _c(w), _c(rbar)
    qbar = np.empty_like(q)
    wbar = np.empty_like(w)
    _check(_load().orc_adjoint(q.shape[1], w.shape[1], _p(e2n), _p(q), _p(w), gamma, _p(rbar),
                               _p(qbar), _p(wbar)), "orc_adjoint")
    return qbar, wbar
