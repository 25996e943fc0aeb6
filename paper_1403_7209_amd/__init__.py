"""Python binding of libopflux, the MI355X edge-flux library.

Argument marshalling only: every step of the path (edge loops, stage updates,
reductions) runs in the library's HIP kernels.  PyTorch supplies device
memory (tensors become the library's borrowed dats) and streams.

The calls mirror the C ABI in include/opflux.h, which follows the OP2 API of
the paper (Sec. 3.1): declare sets, an edge->node map and data on sets, then
run loops over sets whose arguments say how each array is reached and
accessed.
"""
import ctypes
import os

import numpy as np
import torch

from . import _build

__all__ = ["Context", "OpfError", "FluxProblem", "EdgeFluxFunction", "RK_ALPHA", "load",
           "COLOURED", "ATOMIC", "OWNER", "COLOURED_LDS_ATOMIC", "FLAT", "VARIANTS"]

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = _build.LIB

OK, EINVAL, ERANGE, ESIZE, ETYPE, EACCESS, ESTATE, ENOMEM, EDEVICE, ENONFINITE, EPLAN = \
    0, -1, -2, -3, -4, -5, -6, -7, -8, -9, -10
STATUS = {0: "OPF_OK", -1: "OPF_EINVAL", -2: "OPF_ERANGE", -3: "OPF_ESIZE", -4: "OPF_ETYPE",
          -5: "OPF_EACCESS", -6: "OPF_ESTATE", -7: "OPF_ENOMEM", -8: "OPF_EDEVICE",
          -9: "OPF_ENONFINITE", -10: "OPF_EPLAN"}
F64, F32 = 0, 1
READ, WRITE, RW, INC, MIN = 0, 1, 2, 3, 4
(K_EDGE_FLUX, K_EDGE_FLUX_ADJ, K_RK_STAGE, K_EDGE_SPECRAD, K_DT_MIN, K_LOCAL_DT, K_EDGE_GRAD,
 K_EDGE_FLUX2, K_GEOMETRY, K_GEOMETRY_ADJ) = range(10)
COLOURED, ATOMIC, OWNER, COLOURED_LDS_ATOMIC, FLAT = 0, 1, 2, 3, 4
VARIANTS = {"coloured": COLOURED, "atomic": ATOMIC, "owner": OWNER,
            "coloured-lds-atomic": COLOURED_LDS_ATOMIC, "flat": FLAT}
RENUMBER = {"none": 0, "rcm": 1, "morton": 2}
ID = -1
ALL = -2

# Stage coefficients of the 5-stage scheme (low-storage form
# q_k = q_0 - alpha_k dt res(q_{k-1}) / vol).
RK_ALPHA = (1.0 / 4.0, 1.0 / 6.0, 3.0 / 8.0, 1.0 / 2.0, 1.0)

# Exported symbols of include/opflux.h.
SYMBOLS = ("opf_init", "opf_finalize", "opf_last_error", "opf_set_allocator", "opf_decl_set",
           "opf_decl_map", "opf_plan", "opf_get_perm", "opf_plan_view_get", "opf_plan_verify",
           "opf_decl_dat", "opf_par_loop", "opf_edge_flux", "opf_edge_flux_adjoint",
           "opf_edge_specrad", "opf_edge_gradient", "opf_edge_flux2", "opf_rk_stage",
           "opf_rk_stage_local", "opf_local_dt", "opf_dt_min", "opf_edge_flux_stage",
           "opf_edge_flux_stage_noalloc", "opf_geometry",
           "opf_geometry_adjoint",
           "opf_sync", "opf_check_finite")


class OpfError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class PlanOpts(ctypes.Structure):
    _fields_ = [("renumber", ctypes.c_int32), ("block_size", ctypes.c_int32),
                ("colour_sort", ctypes.c_int32), ("cluster_size", ctypes.c_int32),
                ("lane_groups", ctypes.c_int32), ("owner_compact", ctypes.c_int32),
                ("bank_spread", ctypes.c_int32), ("halo_order", ctypes.c_int32),
                ("coords", ctypes.c_void_p)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("nblocks", ctypes.c_int64), ("nblock_colours", ctypes.c_int32),
                ("max_elem_colours", ctypes.c_int32), ("mean_elem_colours", ctypes.c_double),
                ("sum_unique", ctypes.c_int64), ("max_unique", ctypes.c_int32),
                ("min_blocks_per_colour", ctypes.c_int32), ("bandwidth_before", ctypes.c_int64),
                ("bandwidth_after", ctypes.c_int64), ("plan_seconds", ctypes.c_double),
                ("device_bytes", ctypes.c_int64), ("nclusters", ctypes.c_int64),
                ("owner_edge_visits", ctypes.c_int64), ("max_cluster_segments", ctypes.c_int32),
                ("owner_ok", ctypes.c_int32), ("owner_compact", ctypes.c_int32),
                ("flat_colours", ctypes.c_int32),
                ("flat_ok", ctypes.c_int32), ("coloured_ok", ctypes.c_int32)]


class PlanView(ctypes.Structure):
    _fields_ = [("nnodes", ctypes.c_int64), ("nedges", ctypes.c_int64), ("nblocks", ctypes.c_int64),
                ("nblock_colours", ctypes.c_int32), ("block_size", ctypes.c_int32),
                ("e2n", ctypes.c_void_p), ("block_offsets", ctypes.c_void_p),
                ("block_colour", ctypes.c_void_p), ("colour_blocks", ctypes.c_void_p),
                ("colour_offsets", ctypes.c_void_p), ("elem_colour", ctypes.c_void_p),
                ("block_ncolours", ctypes.c_void_p), ("unique_offsets", ctypes.c_void_p),
                ("unique_nodes", ctypes.c_void_p), ("local_idx", ctypes.c_void_p),
                ("cluster_size", ctypes.c_int64), ("nclusters", ctypes.c_int64),
                ("cluster_seg_offsets", ctypes.c_void_p), ("cluster_seg_start", ctypes.c_void_p),
                ("cluster_seg_len", ctypes.c_void_p), ("cluster_range", ctypes.c_void_p),
                ("cluster_list_offsets", ctypes.c_void_p), ("cluster_list_edges", ctypes.c_void_p),
                ("nflat_colours", ctypes.c_int64), ("flat_offsets", ctypes.c_void_p),
                ("flat_edges", ctypes.c_void_p), ("owner_swap", ctypes.c_void_p),
                ("cluster_interior", ctypes.c_void_p), ("cluster_cut_offsets", ctypes.c_void_p),
                ("cluster_cut_edges", ctypes.c_void_p), ("cluster_cut_ends", ctypes.c_void_p),
                ("cluster_cutf_edges", ctypes.c_void_p), ("cluster_cutf_ends", ctypes.c_void_p)]


class PlanReport(ctypes.Structure):
    _fields_ = [("ok", ctypes.c_int32), ("property", ctypes.c_int32), ("where", ctypes.c_int64),
                ("message", ctypes.c_char * 160)]


class Arg(ctypes.Structure):
    _fields_ = [("dat", ctypes.c_int32), ("idx", ctypes.c_int32), ("map", ctypes.c_int32),
                ("dim", ctypes.c_int32), ("type", ctypes.c_int32), ("access", ctypes.c_int32)]


class Gbl(ctypes.Structure):
    _fields_ = [("ptr", ctypes.c_void_p), ("dim", ctypes.c_int32), ("type", ctypes.c_int32),
                ("access", ctypes.c_int32), ("on_device", ctypes.c_int32)]


_lib = None


def _hip_runtimes():
    with open("/proc/self/maps") as f:
        return sorted({ln.split()[-1] for ln in f if "libamdhip64" in ln})


def load():
    """Loads libopflux.so (after torch, so both share torch's HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1403_7209_amd._build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name in SYMBOLS:
        getattr(lib, name)  # raises AttributeError if the export is missing
    vp, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    lib.opf_init.argtypes = [P(vp), ctypes.c_int]
    lib.opf_finalize.argtypes = [vp]
    lib.opf_last_error.argtypes = [vp]
    lib.opf_last_error.restype = ctypes.c_char_p
    lib.opf_set_allocator.argtypes = [vp, vp, vp, vp]
    lib.opf_decl_set.argtypes = [vp, i64, ctypes.c_char_p, P(i32)]
    lib.opf_decl_map.argtypes = [vp, i32, i32, ctypes.c_int, vp, ctypes.c_int, ctypes.c_char_p, P(i32)]
    lib.opf_plan.argtypes = [vp, i32, P(PlanOpts), P(PlanInfo)]
    lib.opf_get_perm.argtypes = [vp, i32, vp]
    lib.opf_plan_view_get.argtypes = [vp, i32, P(PlanView)]
    lib.opf_plan_verify.argtypes = [vp, i32, P(PlanReport)]
    lib.opf_decl_dat.argtypes = [vp, i32, ctypes.c_int, ctypes.c_int, vp, i64, ctypes.c_char_p, P(i32)]
    lib.opf_par_loop.argtypes = [vp, ctypes.c_int, i32, ctypes.c_int, P(Arg), ctypes.c_int, P(Gbl),
                                 ctypes.c_int, vp]
    lib.opf_edge_flux.argtypes = [vp, i32, i32, i32, i32, i32, d, ctypes.c_int, ctypes.c_int, vp]
    lib.opf_edge_flux_adjoint.argtypes = [vp, i32, i32, i32, i32, i32, i32, i32, d, ctypes.c_int,
                                          ctypes.c_int, vp]
    lib.opf_edge_specrad.argtypes = [vp, i32, i32, i32, i32, i32, d, ctypes.c_int, vp]
    lib.opf_edge_gradient.argtypes = [vp, i32, i32, i32, i32, i32, ctypes.c_int, ctypes.c_int, vp]
    lib.opf_edge_flux2.argtypes = [vp, i32, i32, i32, i32, i32, i32, i32, i32, d, ctypes.c_int,
                                   ctypes.c_int, vp]
    lib.opf_rk_stage.argtypes = [vp, i32, i32, i32, i32, i32, d, vp, ctypes.c_int, vp]
    lib.opf_dt_min.argtypes = [vp, i32, i32, i32, d, vp, vp]
    lib.opf_rk_stage_local.argtypes = [vp, i32, i32, i32, i32, i32, i32, d, vp, ctypes.c_int, vp]
    lib.opf_local_dt.argtypes = [vp, i32, i32, i32, d, i32, vp]
    lib.opf_geometry.argtypes = [vp, i32, i32, i32, i32, d, i32, i32, vp]
    lib.opf_edge_flux_stage.argtypes = [vp, i32, i32, i32, i32, i32, i32, i32, i32, d, d, vp, vp]
    lib.opf_edge_flux_stage_noalloc.argtypes = [vp, i32, i32, i32, i32, i32, i32, i32, i32, d, d,
                                                vp, vp]
    lib.opf_geometry_adjoint.argtypes = [vp, i32, i32, i32, i32, d, i32, i32, i32, vp]
    lib.opf_sync.argtypes = [vp, vp]
    lib.opf_check_finite.argtypes = [vp, vp, ctypes.c_int, vp]
    runtimes = _hip_runtimes()
    if len(runtimes) > 1:
        raise RuntimeError(f"more than one HIP runtime is mapped: {runtimes}")
    _lib = lib
    return lib


def _np_ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _stream_ptr(stream, device):
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return ctypes.c_void_p(stream.cuda_stream)


class Context:
    """An opf_ctx bound to one GPU (device >= 0) or host-only (device=None)."""

    def __init__(self, device=None):
        self.lib = load()
        if device is None:
            self.device = -1
        else:
            dev = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
            self.device = dev.index if dev.index is not None else torch.cuda.current_device()
        self._ctx = ctypes.c_void_p()
        rc = self.lib.opf_init(ctypes.byref(self._ctx), self.device)
        if rc:
            raise OpfError(rc, f"opf_init(device={self.device})")
        self._dats = {}
        self._keep = []
        self._problems = 0  # FluxProblems declared on this context (their map names)

    @property
    def torch_device(self):
        return torch.device("cuda", self.device)

    def _check(self, rc, what):
        if rc:
            msg = self.lib.opf_last_error(self._ctx).decode(errors="replace")
            raise OpfError(rc, f"{what}: {msg}")

    def close(self):
        if self._ctx:
            self.lib.opf_finalize(self._ctx)
            self._ctx = ctypes.c_void_p()
            self._dats.clear()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- declarations ------------------------------------------------------
    def decl_set(self, size, name=""):
        out = ctypes.c_int32()
        self._check(self.lib.opf_decl_set(self._ctx, int(size), name.encode(), ctypes.byref(out)),
                    "opf_decl_set")
        return out.value

    def decl_map(self, from_set, to_set, dim, idx, index_base=0, name=""):
        idx = np.ascontiguousarray(idx, dtype=np.int32)
        out = ctypes.c_int32()
        self._check(self.lib.opf_decl_map(self._ctx, from_set, to_set, dim, _np_ptr(idx), index_base,
                                          name.encode(), ctypes.byref(out)), "opf_decl_map")
        return out.value

    def plan(self, m, renumber="rcm", block_size=512, colour_sort=False, coords=None,
             cluster_size=512, lane_groups=True, owner_compact=False, bank_spread=True,
             halo_order=True):
        c = None if coords is None else np.ascontiguousarray(coords, dtype=np.float64)
        opts = PlanOpts(RENUMBER[renumber], block_size, 1 if colour_sort else 0, cluster_size,
                        1 if lane_groups else 0, 1 if owner_compact else 0,
                        1 if bank_spread else 0, 1 if halo_order else 0,
                        None if c is None else c.ctypes.data)
        info = PlanInfo()
        self._check(self.lib.opf_plan(self._ctx, m, ctypes.byref(opts), ctypes.byref(info)),
                    "opf_plan")
        return {k: getattr(info, k) for k, _ in PlanInfo._fields_}

    def get_perm(self, s, size):
        out = np.empty(size, dtype=np.int32)
        self._check(self.lib.opf_get_perm(self._ctx, s, _np_ptr(out)), "opf_get_perm")
        return out

    def plan_view(self, m):
        v = PlanView()
        self._check(self.lib.opf_plan_view_get(self._ctx, m, ctypes.byref(v)), "opf_plan_view_get")
        nb, E, nc = v.nblocks, v.nedges, v.nblock_colours

        def arr(ptr, ctype, n, dtype):
            if n == 0:
                return np.empty(0, dtype=dtype)
            if not ptr:  # an array the plan does not have (no two-level colouring)
                return None
            buf = (ctype * n).from_address(ptr)
            return np.frombuffer(buf, dtype=dtype).copy()

        uoff = arr(v.unique_offsets, ctypes.c_int64, nb + 1, np.int64)
        ncl = v.nclusters
        soff = arr(v.cluster_seg_offsets, ctypes.c_int64, ncl + 1, np.int64) if ncl else \
            np.zeros(1, np.int64)
        nseg = int(soff[-1])
        loff = arr(v.cluster_list_offsets, ctypes.c_int64, ncl + 1, np.int64) if ncl else \
            np.zeros(1, np.int64)
        coff = arr(v.cluster_cut_offsets, ctypes.c_int64, ncl + 1, np.int64) if ncl else \
            np.zeros(1, np.int64)
        return dict(nnodes=v.nnodes, nedges=E, nblocks=nb, nblock_colours=nc,
                    cluster_size=v.cluster_size, nclusters=ncl, cluster_seg_offsets=soff,
                    cluster_seg_start=arr(v.cluster_seg_start, ctypes.c_int32, nseg, np.int32),
                    cluster_seg_len=arr(v.cluster_seg_len, ctypes.c_int32, nseg, np.int32),
                    cluster_range=arr(v.cluster_range, ctypes.c_int32, 2 * ncl,
                                      np.int32).reshape(ncl, 2),
                    cluster_list_offsets=loff,
                    cluster_list_edges=arr(v.cluster_list_edges, ctypes.c_int32, int(loff[-1]),
                                           np.int32),
                    block_size=v.block_size,
                    e2n=arr(v.e2n, ctypes.c_int32, 2 * E, np.int32).reshape(E, 2),
                    block_offsets=arr(v.block_offsets, ctypes.c_int64, nb + 1, np.int64),
                    block_colour=arr(v.block_colour, ctypes.c_int32, nb, np.int32),
                    colour_blocks=arr(v.colour_blocks, ctypes.c_int32, nb, np.int32),
                    colour_offsets=arr(v.colour_offsets, ctypes.c_int64, nc + 1, np.int64),
                    elem_colour=arr(v.elem_colour, ctypes.c_uint8, E, np.uint8),
                    block_ncolours=arr(v.block_ncolours, ctypes.c_int32, nb, np.int32),
                    unique_offsets=uoff,
                    unique_nodes=None if uoff is None else
                    arr(v.unique_nodes, ctypes.c_int32, int(uoff[-1]), np.int32),
                    local_idx=None if not v.local_idx else
                    arr(v.local_idx, ctypes.c_uint16, 2 * E, np.uint16).reshape(E, 2),
                    nflat_colours=v.nflat_colours,
                    flat_offsets=arr(v.flat_offsets, ctypes.c_int64, v.nflat_colours + 1,
                                     np.int64) if v.nflat_colours else None,
                    flat_edges=arr(v.flat_edges, ctypes.c_int32, E, np.int32)
                    if v.nflat_colours else None,
                    owner_swap=arr(v.owner_swap, ctypes.c_uint8, E, np.uint8)
                    if v.owner_swap else None,
                    cluster_interior=arr(v.cluster_interior, ctypes.c_int32, ncl, np.int32)
                    if ncl else np.zeros(0, np.int32),
                    cluster_cut_offsets=coff,
                    cluster_cut_edges=arr(v.cluster_cut_edges, ctypes.c_int32, int(coff[-1]),
                                          np.int32),
                    cluster_cut_ends=arr(v.cluster_cut_ends, ctypes.c_uint8, int(coff[-1]),
                                         np.uint8),
                    cluster_cutf_edges=arr(v.cluster_cutf_edges, ctypes.c_int32, int(coff[-1]),
                                           np.int32),
                    cluster_cutf_ends=arr(v.cluster_cutf_ends, ctypes.c_uint8, int(coff[-1]),
                                          np.uint8))

    def plan_verify(self, m):
        rep = PlanReport()
        rc = self.lib.opf_plan_verify(self._ctx, m, ctypes.byref(rep))
        if rc not in (OK, EPLAN):
            self._check(rc, "opf_plan_verify")
        return dict(ok=bool(rep.ok), property=rep.property, where=rep.where,
                    message=rep.message.decode(errors="replace"), status=rc)

    def decl_dat(self, s, tensor, name=""):
        """Declares a dat on set s borrowing a (dim, ld) or (ld,) device tensor."""
        t = tensor
        if t.dim() == 1:
            dim, ld = 1, t.shape[0]
        elif t.dim() == 2:
            dim, ld = t.shape[0], t.stride(0)
            if t.stride(1) != 1:
                raise ValueError("dat tensors must be contiguous along elements")
        else:
            raise ValueError("dat tensors are (dim, ld) or (ld,)")
        if t.dtype == torch.float64:
            typ = F64
        elif t.dtype == torch.float32:
            typ = F32
        else:
            raise TypeError(f"unsupported dat dtype {t.dtype}")
        if self.device >= 0 and (not t.is_cuda or t.device.index != self.device):
            raise ValueError(f"dat '{name}' must be a tensor on cuda:{self.device}")
        key = (s, t.data_ptr(), dim, typ, ld)
        if key in self._dats:
            return self._dats[key]
        out = ctypes.c_int32()
        self._check(self.lib.opf_decl_dat(self._ctx, s, dim, typ, ctypes.c_void_p(t.data_ptr()), ld,
                                          name.encode(), ctypes.byref(out)), "opf_decl_dat")
        self._dats[key] = out.value
        return out.value

    # -- loops -----------------------------------------------------------------
    def _gbl_ptr(self, t, n, what):
        """Device address of a float64 global of at least n values on this
        context's GPU (a host tensor would hand the kernel a host address)."""
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{what} must be a torch tensor")
        if self.device < 0 or not t.is_cuda or t.device.index != self.device:
            raise ValueError(f"{what} must be a tensor on cuda:{self.device}")
        if t.dtype != torch.float64:
            raise TypeError(f"{what} must be float64")
        if t.numel() < n or not t.is_contiguous():
            raise ValueError(f"{what} must be contiguous with at least {n} values")
        return ctypes.c_void_p(t.data_ptr())

    def par_loop(self, kernel, s, args, gbls, variant=COLOURED, stream=None):
        a = (Arg * len(args))(*[Arg(*x) for x in args])
        g = (Gbl * len(gbls))(*[Gbl(*x) for x in gbls])
        self._check(self.lib.opf_par_loop(self._ctx, kernel, s, len(args), a, len(gbls), g, variant,
                                          _stream_ptr(stream, self.device)), "opf_par_loop")

    def edge_flux(self, edges, e2n, q, n, res, gamma=1.4, variant=COLOURED, res_access=INC,
                  stream=None):
        """res_access INC (res += sum), or WRITE (res = sum; OWNER variant only)."""
        self._check(self.lib.opf_edge_flux(self._ctx, edges, e2n, q, n, res, gamma, variant,
                                           res_access, _stream_ptr(stream, self.device)),
                    "opf_edge_flux")

    def edge_flux_adjoint(self, edges, e2n, q, n, rbar, qbar, nbar, gamma=1.4, variant=COLOURED,
                          qbar_access=INC, stream=None):
        self._check(self.lib.opf_edge_flux_adjoint(self._ctx, edges, e2n, q, n, rbar, qbar, nbar,
                                                   gamma, variant, qbar_access,
                                                   _stream_ptr(stream, self.device)),
                    "opf_edge_flux_adjoint")

    def edge_specrad(self, edges, e2n, q, n, lam, gamma=1.4, variant=COLOURED, stream=None):
        self._check(self.lib.opf_edge_specrad(self._ctx, edges, e2n, q, n, lam, gamma, variant,
                                              _stream_ptr(stream, self.device)), "opf_edge_specrad")

    def edge_gradient(self, edges, e2n, q, n, G, variant=COLOURED, g_access=INC, stream=None):
        """Green-Gauss sums G (18 per node, component 3v + d) += over the edges."""
        self._check(self.lib.opf_edge_gradient(self._ctx, edges, e2n, q, n, G, variant, g_access,
                                               _stream_ptr(stream, self.device)),
                    "opf_edge_gradient")

    def edge_flux2(self, edges, e2n, q, G, vol, n, dx, res, gamma=1.4, variant=COLOURED,
                   res_access=INC, stream=None):
        """Second-order residual from the Green-Gauss sums G and edge vectors dx."""
        self._check(self.lib.opf_edge_flux2(self._ctx, edges, e2n, q, G, vol, n, dx, res, gamma,
                                            variant, res_access, _stream_ptr(stream, self.device)),
                    "opf_edge_flux2")

    def edge_flux_stage(self, edges, e2n, q, n, q0, vol, qout, alpha, ss, gamma=1.4, dt=-1,
                        stream=None):
        """Owner edge-flux loop with the stage update fused: qout = q0 - alpha res/vol
        (alpha dt_i res/vol with a per-node step dat), ss += sum res^2."""
        self._check(self.lib.opf_edge_flux_stage(self._ctx, edges, e2n, q, n, q0, vol, dt, qout,
                                                 gamma, float(alpha), self._gbl_ptr(ss, 6, "ss"),
                                                 _stream_ptr(stream, self.device)),
                    "opf_edge_flux_stage")

    def edge_flux_stage_noalloc(self, edges, e2n, q, n, q0, vol, qout, alpha, ss, gamma=1.4,
                                dt=-1, stream=None):
        """edge_flux_stage through the allocation-free entry point (partial sums in
        the library's static device scratch; calls overlapping on one GPU race)."""
        self._check(self.lib.opf_edge_flux_stage_noalloc(self._ctx, edges, e2n, q, n, q0, vol, dt,
                                                         qout, gamma, float(alpha),
                                                         self._gbl_ptr(ss, 6, "ss"),
                                                         _stream_ptr(stream, self.device)),
                    "opf_edge_flux_stage_noalloc")

    def geometry(self, tets, t2n, t2e, x, w, vol, period=1.0, variant=OWNER, stream=None,
                 access=INC):
        """w (edge dat, 3) and vol (node dat) += median-dual weights and volumes of the
        tets (OWNER: gather over incident tets, deterministic; ATOMIC: scatter).
        access=WRITE (OWNER only) overwrites them instead."""
        if access == INC:
            self._check(self.lib.opf_geometry(self._ctx, tets, t2n, t2e, x, float(period), w, vol,
                                              variant, _stream_ptr(stream, self.device)),
                        "opf_geometry")
            return
        per = ctypes.c_double(period)
        self.par_loop(K_GEOMETRY, tets,
                      [(x, ALL, t2n, 3, F64, READ), (w, ALL, t2e, 3, F64, access),
                       (vol, ALL, t2n, 1, F64, access)],
                      [(ctypes.addressof(per), 1, F64, READ, 0)],
                      variant, stream)

    def geometry_adjoint(self, tets, t2n, t2e, x, wbar, volbar, xbar, period=1.0, variant=OWNER,
                         stream=None):
        """xbar (node dat, 3) += (dw/dx)^T wbar + (dvol/dx)^T volbar."""
        self._check(self.lib.opf_geometry_adjoint(self._ctx, tets, t2n, t2e, x, float(period),
                                                  wbar, volbar, xbar, variant,
                                                  _stream_ptr(stream, self.device)),
                    "opf_geometry_adjoint")

    def rk_stage(self, nodes, q0, res, vol, q, alpha_dt, ss, res_access=RW, stream=None):
        """ss: float64 device tensor of 6 values, incremented by sum res^2.
        res_access RW zeroes res after use, READ leaves it."""
        self._check(self.lib.opf_rk_stage(self._ctx, nodes, q0, res, vol, q, float(alpha_dt),
                                          self._gbl_ptr(ss, 6, "ss"), res_access,
                                          _stream_ptr(stream, self.device)), "opf_rk_stage")

    def rk_stage_local(self, nodes, q0, res, vol, dt, q, alpha, ss, res_access=RW, stream=None):
        """As rk_stage with a time step per node (dat dt): q = q0 - alpha dt_i res / vol."""
        self._check(self.lib.opf_rk_stage_local(self._ctx, nodes, q0, res, vol, dt, q, float(alpha),
                                                self._gbl_ptr(ss, 6, "ss"), res_access,
                                                _stream_ptr(stream, self.device)),
                    "opf_rk_stage_local")

    def local_dt(self, nodes, vol, lam, cfl, dt, stream=None):
        """dt_i = cfl vol_i / lam_i (dats on the node set)."""
        self._check(self.lib.opf_local_dt(self._ctx, nodes, vol, lam, float(cfl), dt,
                                          _stream_ptr(stream, self.device)), "opf_local_dt")

    def dt_min(self, nodes, vol, lam, cfl, dt, stream=None):
        self._check(self.lib.opf_dt_min(self._ctx, nodes, vol, lam, float(cfl),
                                        self._gbl_ptr(dt, 1, "dt"),
                                        _stream_ptr(stream, self.device)), "opf_dt_min")

    def sync(self, stream=None):
        self._check(self.lib.opf_sync(self._ctx, _stream_ptr(stream, self.device)), "opf_sync")

    def check_finite(self, t, stream=None):
        rc = self.lib.opf_check_finite(self._ctx, self._gbl_ptr(t, 1, "t"), t.numel(),
                                       _stream_ptr(stream, self.device))
        if rc == ENONFINITE:
            return False
        self._check(rc, "opf_check_finite")
        return True


class FluxProblem:
    """The edge-flux path on one mesh: node and edge sets, the edge->node map,
    its plan, and device dats in the library's internal numbering.

    Inputs are host arrays in user numbering: e2n (E, 2) int32, w (3, E)
    weights, vol (N,), q (6, N).  fp32=True keeps the state and weights in
    FP32 (the residual, volumes and reductions stay FP64)."""

    def __init__(self, ctx, e2n, w, vol, q, fp32=False, renumber="rcm", block_size=512,
                 colour_sort=False, coords=None, gamma=1.4, index_base=0, like=None,
                 cluster_size=512, lane_groups=True, tets=None, tet_edges=None,
                 owner_compact=False, bank_spread=True, halo_order=True):
        self.ctx, self.gamma, self.fp32 = ctx, float(gamma), fp32
        if like is not None:  # same mesh, sets, map and plan; other dats
            if like.ctx is not ctx:
                raise ValueError("like= must be a problem on the same context")
            for k in ("N", "E", "nodes", "edges", "e2n", "info", "node_new", "edge_new", "tets",
                      "t2n", "t2e"):
                setattr(self, k, getattr(like, k))
        else:
            e2n = np.ascontiguousarray(e2n, dtype=np.int32)
            self.N, self.E = int(np.asarray(vol).shape[0]), int(e2n.shape[0])
            # a map declared under a name already taken replaces that map, so
            # every problem on a context names its maps apart
            ctx._problems += 1
            tag = f"/{ctx._problems}"
            self.nodes = ctx.decl_set(self.N, "nodes" + tag)
            self.edges = ctx.decl_set(self.E, "edges" + tag)
            self.e2n = ctx.decl_map(self.edges, self.nodes, 2, e2n, index_base, "e2n" + tag)
            self.tets = self.t2n = self.t2e = None
            if tets is not None:  # tet maps must exist before the plan renumbers the sets
                tets = np.ascontiguousarray(tets, dtype=np.int32)
                self.tets = ctx.decl_set(tets.shape[0], "tets" + tag)
                self.t2n = ctx.decl_map(self.tets, self.nodes, 4, tets, index_base, "t2n" + tag)
                self.t2e = ctx.decl_map(self.tets, self.edges, 6,
                                        np.ascontiguousarray(tet_edges, dtype=np.int32),
                                        index_base, "t2e" + tag)
            self.info = ctx.plan(self.e2n, renumber=renumber, block_size=block_size,
                                 colour_sort=colour_sort, coords=coords,
                                 cluster_size=cluster_size, lane_groups=lane_groups,
                                 owner_compact=owner_compact, bank_spread=bank_spread,
                                 halo_order=halo_order)
            self.node_new = ctx.get_perm(self.nodes, self.N)
            self.edge_new = ctx.get_perm(self.edges, self.E)
        dev = ctx.torch_device
        self.tdtype = torch.float32 if fp32 else torch.float64
        self.w_t = self.nodes_in(w, edges=True).to(self.tdtype)
        self.vol_t = self.nodes_in(np.asarray(vol, dtype=np.float64)[None, :])[0].contiguous()
        self.qa = self.nodes_in(q).to(self.tdtype)          # q0 / state
        self.qb = torch.empty_like(self.qa)                  # stage state
        self.res = torch.zeros((6, self.N), dtype=torch.float64, device=dev)
        self.ss = torch.zeros((5, 6), dtype=torch.float64, device=dev)
        self.lam = torch.zeros(self.N, dtype=torch.float64, device=dev)
        self.dt_t = torch.full((1,), float("inf"), dtype=torch.float64, device=dev)
        self.w = ctx.decl_dat(self.edges, self.w_t, "n")
        self.vol = ctx.decl_dat(self.nodes, self.vol_t, "vol")
        self.res_d = ctx.decl_dat(self.nodes, self.res, "res")
        self.lam_d = ctx.decl_dat(self.nodes, self.lam, "lam")

    # -- numbering -------------------------------------------------------------
    def nodes_in(self, a, edges=False):
        """Host (d, n) array in user numbering -> device tensor in internal numbering."""
        a = np.asarray(a)
        perm = self.edge_new if edges else self.node_new
        out = np.empty(a.shape, dtype=a.dtype)  # C order whatever the layout of a
        out[:, perm] = a
        return torch.from_numpy(out).to(self.ctx.torch_device)

    def nodes_out(self, t, edges=False):
        """Device tensor in internal numbering -> host array in user numbering."""
        perm = self.edge_new if edges else self.node_new
        return t.detach().cpu().numpy()[:, perm]

    def dat(self, t, name="", edges=False):
        return self.ctx.decl_dat(self.edges if edges else self.nodes, t, name)

    # -- loops -------------------------------------------------------------------
    def residual(self, q_t, res_t, variant=COLOURED, res_access=INC, stream=None):
        """res_t += edge-flux residual of state q_t (both internal numbering);
        res_access=WRITE (OWNER variant) overwrites instead."""
        self.ctx.edge_flux(self.edges, self.e2n, self.dat(q_t, "q"), self.w, self.dat(res_t, "res"),
                           self.gamma, variant, res_access, stream)

    def compute_dt(self, cfl=0.5, variant=COLOURED, stream=None):
        """Global time step cfl * min_i vol_i / sum_e lambda_e of the current state."""
        self.lam.zero_()
        self.dt_t.fill_(float("inf"))
        self.ctx.edge_specrad(self.edges, self.e2n, self.dat(self.qa, "q"), self.w, self.lam_d,
                              self.gamma, variant, stream)
        self.ctx.dt_min(self.nodes, self.vol, self.lam_d, cfl, self.dt_t, stream)
        return float(self.dt_t.item())

    def _rk_fused(self, alpha_of_stage, dt_dat, stream):
        """Five stages of the owner loop with the update fused in; stage k reads
        the state of stage k-1 and writes the other of two stage buffers."""
        if not hasattr(self, "qc"):
            self.qc = torch.empty_like(self.qa)
        qa = self.dat(self.qa, "qa")
        bufs = (self.dat(self.qb, "qb"), self.dat(self.qc, "qc"))
        self.ss.zero_()
        src = qa
        for k in range(5):
            dst = bufs[k % 2]
            self.ctx.edge_flux_stage(self.edges, self.e2n, src, self.w, qa, self.vol, dst,
                                     alpha_of_stage(k), self.ss[k], self.gamma, dt_dat, stream)
            src = dst
        # stage 5 wrote qb (k = 4 -> bufs[0])
        self.qa, self.qb = self.qb, self.qa

    def rk_iteration(self, dt, variant=COLOURED, stream=None, fused=True):
        """One 5-stage iteration; the new state is left in self.qa.  self.ss
        (5, 6) receives each stage's per-variable sum of squared residuals.
        With the OWNER variant the stage update is fused into the edge loop
        unless fused=False."""
        if variant == OWNER and fused:
            return self._rk_fused(lambda k: RK_ALPHA[k] * dt, -1, stream)
        qa, qb = self.dat(self.qa, "qa"), self.dat(self.qb, "qb")
        # the owner variant writes each residual once: no zeroing pass needed
        ra, rk = (WRITE, READ) if variant == OWNER else (INC, RW)
        self.ss.zero_()
        for k in range(5):
            src = qa if k == 0 else qb
            self.ctx.edge_flux(self.edges, self.e2n, src, self.w, self.res_d, self.gamma, variant,
                               ra, stream)
            self.ctx.rk_stage(self.nodes, qa, self.res_d, self.vol, qb, RK_ALPHA[k] * dt,
                              self.ss[k], rk, stream)
        self.qa, self.qb = self.qb, self.qa

    def geometry(self, x_t, w_t, vol_t, period=1.0, variant=OWNER, stream=None, access=INC):
        """w_t (3, E) and vol_t (N,) += weights and volumes of the tets at node
        coordinates x_t (3, N); all internal numbering, FP64.  access=WRITE
        (OWNER only) overwrites them."""
        self.ctx.geometry(self.tets, self.t2n, self.t2e, self.dat(x_t, "x"),
                          self.dat(w_t, "w", edges=True), self.dat(vol_t[None], "vol_out"),
                          period, variant, stream, access)

    def geometry_adjoint(self, x_t, wbar_t, volbar_t, xbar_t, period=1.0, variant=OWNER,
                         stream=None):
        self.ctx.geometry_adjoint(self.tets, self.t2n, self.t2e, self.dat(x_t, "x"),
                                  self.dat(wbar_t, "wbar", edges=True),
                                  self.dat(volbar_t[None], "volbar"), self.dat(xbar_t, "xbar"),
                                  period, variant, stream)

    def shape_gradient(self, x_t, rbar_t, period=1.0, variant=COLOURED, stream=None):
        """d(rbar . R(q, w(x)))/dx at the current state (FP64): the flux adjoint
        gives the weight sensitivities, the geometry reverse carries them to the
        node coordinates.  Returns xbar (3, N), internal numbering."""
        dev = self.ctx.torch_device
        qbar = torch.zeros((6, self.N), dtype=torch.float64, device=dev)
        nbar = torch.empty((3, self.E), dtype=torch.float64, device=dev)
        self.ctx.edge_flux_adjoint(self.edges, self.e2n, self.dat(self.qa, "q"), self.w,
                                   self.dat(rbar_t, "rbar"), self.dat(qbar, "qbar"),
                                   self.dat(nbar, "nbar", edges=True), self.gamma, variant, INC,
                                   stream)
        xbar = torch.zeros((3, self.N), dtype=torch.float64, device=dev)
        volbar = torch.zeros(self.N, dtype=torch.float64, device=dev)
        self.geometry_adjoint(x_t, nbar, volbar, xbar, period, OWNER, stream)
        return xbar

    def set_edge_vectors(self, dx):
        """Edge vectors x_j - x_i (3, E), user numbering, for the second-order loop."""
        self.dx_t = self.nodes_in(np.asarray(dx, dtype=np.float64), edges=True)
        self.dx = self.ctx.decl_dat(self.edges, self.dx_t, "dx")

    def gradient(self, q_t, G_t, variant=COLOURED, g_access=INC, stream=None):
        """G_t (18, N) float64 (internal numbering) += Green-Gauss sums of q_t."""
        self.ctx.edge_gradient(self.edges, self.e2n, self.dat(q_t, "q"), self.w,
                               self.dat(G_t, "G"), variant, g_access, stream)

    def residual2(self, q_t, G_t, res_t, variant=COLOURED, res_access=INC, stream=None):
        """res_t += second-order residual of q_t from its Green-Gauss sums G_t."""
        self.ctx.edge_flux2(self.edges, self.e2n, self.dat(q_t, "q"), self.dat(G_t, "G"), self.vol,
                            self.w, self.dx, self.dat(res_t, "res"), self.gamma, variant,
                            res_access, stream)

    def compute_local_dt(self, cfl=0.5, variant=COLOURED, stream=None):
        """Per-node time steps cfl * vol_i / sum_e lambda_e of the current state,
        left in self.dtl (internal numbering)."""
        if not hasattr(self, "dtl"):
            self.dtl = torch.empty(self.N, dtype=torch.float64, device=self.qa.device)
            self.dtl_d = self.ctx.decl_dat(self.nodes, self.dtl, "dt_local")
        self.lam.zero_()
        self.ctx.edge_specrad(self.edges, self.e2n, self.dat(self.qa, "q"), self.w, self.lam_d,
                              self.gamma, variant, stream)
        self.ctx.local_dt(self.nodes, self.vol, self.lam_d, cfl, self.dtl_d, stream)
        return self.dtl

    def rk_iteration_local(self, variant=COLOURED, stream=None, fused=True):
        """One 5-stage iteration with the per-node steps of the last
        compute_local_dt; otherwise as rk_iteration."""
        if variant == OWNER and fused:
            return self._rk_fused(lambda k: RK_ALPHA[k], self.dtl_d, stream)
        qa, qb = self.dat(self.qa, "qa"), self.dat(self.qb, "qb")
        ra, rk = (WRITE, READ) if variant == OWNER else (INC, RW)
        self.ss.zero_()
        for k in range(5):
            src = qa if k == 0 else qb
            self.ctx.edge_flux(self.edges, self.e2n, src, self.w, self.res_d, self.gamma, variant,
                               ra, stream)
            self.ctx.rk_stage_local(self.nodes, qa, self.res_d, self.vol, self.dtl_d, qb,
                                    RK_ALPHA[k], self.ss[k], rk, stream)
        self.qa, self.qb = self.qb, self.qa

    def rms(self):
        """Per-stage, per-variable RMS sqrt(ss / N) of the last iteration (host)."""
        return np.sqrt(self.ss.cpu().numpy() / self.N)


class EdgeFluxFunction(torch.autograd.Function):
    """res = R(q, n) on a FluxProblem (internal numbering, FP64).  The backward
    pass runs the hand-written adjoint edge kernel, which recomputes the edge
    fluxes instead of storing them."""

    @staticmethod
    def forward(ctx, problem, q, w, variant=COLOURED):
        res = torch.zeros((6, problem.N), dtype=torch.float64, device=q.device)
        problem.ctx.edge_flux(problem.edges, problem.e2n, problem.dat(q.detach(), "q"),
                              problem.dat(w.detach(), "n", edges=True), problem.dat(res, "res"),
                              problem.gamma, variant)
        ctx.problem, ctx.variant = problem, variant
        ctx.save_for_backward(q, w)
        return res

    @staticmethod
    def backward(ctx, rbar):
        q, w = ctx.saved_tensors
        p = ctx.problem
        rbar = rbar.contiguous()
        qbar = torch.zeros_like(q)
        nbar = torch.empty_like(w)
        p.ctx.edge_flux_adjoint(p.edges, p.e2n, p.dat(q.detach(), "q"),
                                p.dat(w.detach(), "n", edges=True), p.dat(rbar, "rbar"),
                                p.dat(qbar, "qbar"), p.dat(nbar, "nbar", edges=True), p.gamma,
                                ctx.variant)
        return None, qbar, nbar, None
