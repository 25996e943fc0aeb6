"""Throughput of the edge-flux hot path on one MI355X.

Workload: the periodic 160^3 box (4,096,000 nodes) split into a layered mix of
5- and 6-tet cubes (26,624,000 edges), nodes jittered by U(-0.25h, 0.25h) and
randomly relabelled, then renumbered by the planner.  All inputs are seeded
and synthetic.  `--mesh B` runs the same step on the 1,000,000-node 100^3 box
of 6-tet cubes jittered by U(-0.2h, 0.2h), `--mesh A` on the 8,000-node 20^3
box of 6-tet cubes without jitter.

One step = one 5-stage Runge-Kutta iteration in FP64 (5 edge-flux loops + 5
stage updates with residual norms), the same iteration in the FP32-storage
form, and one FP64 adjoint edge sweep: 11 edge loops over all edges.  With the
owner variant (the default) each stage update is fused into its edge loop
(opf_edge_flux_stage); other variants run the two loops separately.

value = 11 * E / (seconds per step): edges per second over the whole step,
inputs resident in HBM.  The roofline entry is the dominant kernel: the fused
FP64 edge-flux + stage loop, priced in algorithmic bytes (32 B per edge: map 8
+ weights 24; 152 B per node: state 48 + stage base 48 + volume 8 read, new
state 48 written), or for other variants the FP64 edge-flux loop (32 B per
edge; 96 B per node: state read 48 + residual write 48), against 8 TB/s.

After the timed steps it also times, outside `value`, the Green-Gauss
gradient loop, the second-order edge loop, the local time-step loop and the
tet geometry loop with its reverse (reported under "forms").

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES = {  # algorithmic bytes: (per edge, per node[, per tet])
    "fp64": (32, 96),
    "fp32": (20, 72),
    # the owner loop with the stage update fused in: q read 48 + q0 48 + vol 8 + q
    # written 48 per node (FP32 storage: 24 + 24 + 8 + 24); no residual traffic
    "fp64_fused": (32, 152),
    "fp32_fused": (20, 80),
    "adjoint": (56, 144),
    "rk64": (0, 152),
    "rk32": (0, 104),
    # loops outside the step, timed beside it
    "grad": (32, 192),    # map 8 + n 24; q 48 + G 144 (written)
    "flux2": (56, 248),   # map 8 + n 24 + dx 24; q 48 + G 144 + vol 8 + res 48
    "local_dt": (0, 24),  # vol, lam read; dt written
    # per tet: t2n 16 + t2e 24; per edge: weights written 24; per node: x 24 + vol written 8
    "geometry": (24, 32, 40),
    # per tet: maps 40; per edge: wbar 24; per node: x 24 + volbar 8 + xbar written 24
    "geometry_adj": (24, 56, 40),
    "geometry_atomic": (24, 32, 40),
    "geometry_adj_atomic": (24, 56, 40),
}


# the sources that decide the dominant kernel's traffic: its code and the plan
TRAFFIC_SOURCES = [os.path.join(ROOT, "paper_1403_7209_amd", "csrc", f)
                   for f in ("kernels.hip", "planner.cpp")]
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "edge_flux_fp64_owner_E_traffic.txt")
MESHES = {  # name: (nodes per axis, split, jitter / h, description)
    "E": (160, 1, 0.25, "layered 5/6-tet mix"),
    "B": (100, 0, 0.2, "6 tets per cube"),
    "A": (20, 0, 0.0, "6 tets per cube"),
}


def sources_sha():
    h = hashlib.sha256()
    for path in TRAFFIC_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(config_key):
    """HBM bytes per FP64 edge-flux launch from the committed rocprofv3 counter
    summary, or None when the kernels changed since it was taken or it was
    taken on another launch configuration."""
    try:
        with open(TRAFFIC_PROFILE) as f:
            kv = dict(ln.split(":", 1) for ln in f if ":" in ln and not ln.startswith("#"))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("sources_sha256") != sources_sha() or kv.get("config") != config_key:
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def host_cpu():
    """The host's CPU model name (from /proc/cpuinfo) and its logical CPU count."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline(mesh, q, gpu_res=None, seconds=12.0):
    """The oracle (single thread) on a bounded sample of the same workload:
    repeated FP64 residual passes over the full mesh until ~`seconds` elapse,
    in the input's own (randomly permuted) node numbering, which is what the
    oracle is given; it does not renumber.  gpu_res: {form: residual of the
    same state from the GPU, user numbering}; each is reported with its error
    against the oracle's residual (largest over the six variables of
    max |r - r*| / max |r*|)."""
    import oracle
    passes, t0 = 0, time.perf_counter()
    res = np.zeros_like(q)
    while True:
        res[:] = 0.0
        oracle.residual(mesh.e2n, q, mesh.w, res=res)
        passes += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    model, nproc = host_cpu()
    out = {"value": passes * mesh.E / el, "unit": "edges/s", "cores": 1, "kind": "oracle",
           "host_cpu": model, "host_nproc": nproc,
           "sample": f"{passes} sequential FP64 residual passes over all {mesh.E} edges "
                     f"of the same mesh in its input (randomly permuted) numbering "
                     f"({el:.1f} s, one thread of {nproc})"}
    if gpu_res:
        scale = np.abs(res).max(axis=1)
        out["gpu_residual_error_vs_oracle"] = {
            k: float(f"{float((np.abs(v - res).max(axis=1) / scale).max()):.3e}")
            for k, v in gpu_res.items()}
    return out


def cpu_baseline_sweep():
    """The oracle (single thread) on the host: the FP64 residual and the RK
    stage on the 8,000-node, 1M-node and 4.1M-node meshes, and the adjoint on
    the 1M-node mesh; the best of three runs of each, as edges/s (nodes/s for
    the stage)."""
    import platform

    import meshgen
    import oracle

    def best(fn, reps=3):
        t = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            t.append(time.perf_counter() - t0)
        return min(t)

    out = {"kind": "oracle", "cores": 1, "host": platform.processor() or platform.machine(),
           "nproc": os.cpu_count(), "rows": []}
    for name, (n, split, jit) in (("A", (20, 0, 0.0)), ("B", (100, 0, 0.2)),
                                  ("E", (160, 1, 0.25))):
        mesh = meshgen.build_mesh(n, split, jit)
        q = meshgen.state(mesh.N, mesh.perm)
        res = np.zeros_like(q)
        t = best(lambda: oracle.residual(mesh.e2n, q, mesh.w, res=res))
        out["rows"].append({"mesh": name, "N": mesh.N, "E": mesh.E, "loop": "FP64 residual",
                            "s": round(t, 4), "edges_per_s": round(mesh.E / t, 1)})
        r = np.ascontiguousarray(res)
        t = best(lambda: oracle.rk_stage(q, r, mesh.vol, 1e-4))
        out["rows"].append({"mesh": name, "N": mesh.N, "E": mesh.E, "loop": "RK stage + norms",
                            "s": round(t, 4), "nodes_per_s": round(mesh.N / t, 1)})
        if name == "B":
            rbar = meshgen.normal(6 * mesh.N, purpose=21).reshape(6, mesh.N)
            t = best(lambda: oracle.adjoint(mesh.e2n, q, mesh.w, rbar), reps=1)
            out["rows"].append({"mesh": name, "N": mesh.N, "E": mesh.E,
                                "loop": "FP64 adjoint (dual numbers)", "s": round(t, 4),
                                "edges_per_s": round(mesh.E / t, 1)})
        log(f"oracle on {name}: {out['rows'][-1]}")
    return out


def shard_share(pk, ctx, mesh, q, n, dt, rbar_user, res_user, ev, reps=3):
    """One GPU's share of the mesh split into 2x2x2 blocks: the central block's
    owned nodes, their halo and every edge with an owned end (owner-compute),
    planned as a mesh of its own.  Times its fused FP64 and FP32 iterations and
    its adjoint, and checks its owned residuals against the whole mesh's."""
    import torch

    from paper_1403_7209_amd.shard import lattice_block, owner_shard
    sh = owner_shard(mesh.e2n, lattice_block(mesh.xyz, n, n // 4, n // 2))
    w_s = np.ascontiguousarray(mesh.w[:, sh.edges])
    q_s = np.ascontiguousarray(q[:, sh.nodes])
    ps = pk.FluxProblem(ctx, sh.e2n, w_s, mesh.vol[sh.nodes], q_s, renumber="morton",
                        coords=np.ascontiguousarray(mesh.xyz[:, sh.nodes]))
    ps32 = pk.FluxProblem(ctx, sh.e2n, w_s, mesh.vol[sh.nodes], q_s, fp32=True, like=ps)
    Ns, Es = len(sh.nodes), len(sh.edges)
    dev = ps.qa.device
    rb = ps.nodes_in(np.ascontiguousarray(rbar_user[:, sh.nodes]))
    qbar = torch.zeros((6, Ns), dtype=torch.float64, device=dev)
    nbar = torch.empty((3, Es), dtype=torch.float64, device=dev)
    rb_d, qbar_d, nbar_d = ps.dat(rb, "rbar"), ps.dat(qbar, "qbar"), ps.dat(nbar, "nbar", edges=True)
    for p in (ps, ps32):
        p.qc = torch.empty_like(p.qa)
    timers = {"fp64_fused": [], "fp32_fused": [], "adjoint": []}

    def iteration(p, key, rec):  # five fused stages from the same starting state
        qa = p.dat(p.qa, "qa")
        bufs, src = (p.dat(p.qb, "qb"), p.dat(p.qc, "qc")), qa
        for k in range(5):
            a = ev()
            p.ctx.edge_flux_stage(p.edges, p.e2n, src, p.w, qa, p.vol, bufs[k % 2],
                                  pk.RK_ALPHA[k] * dt, p.ss[k], p.gamma)
            b = ev()
            if rec:
                timers[key].append((a, b))
            src = bufs[k % 2]

    for rec in [False] + [True] * reps:
        iteration(ps, "fp64_fused", rec)
        iteration(ps32, "fp32_fused", rec)
        a = ev()
        ctx.edge_flux_adjoint(ps.edges, ps.e2n, ps.dat(ps.qa, "q"), ps.w, rb_d, qbar_d, nbar_d,
                              ps.gamma, pk.OWNER, pk.WRITE)
        b = ev()
        if rec:
            timers["adjoint"].append((a, b))
    res = torch.empty((6, Ns), dtype=torch.float64, device=dev)
    ps.residual(ps.qa, res, pk.OWNER, pk.WRITE)
    torch.cuda.synchronize()
    own = ps.nodes_out(res)[:, :sh.n_owned]
    ref = res_user[:, sh.nodes[:sh.n_owned]]
    err = float((np.abs(own - ref).max(axis=1) / np.abs(ref).max(axis=1)).max())
    forms = {}
    for k, lst in timers.items():
        ms = float(np.mean([a.elapsed_time(b) for a, b in lst]))
        be, bn = BYTES[k]
        gbs = (be * Es + bn * Ns) / (ms * 1e-3) / 1e9
        forms[k] = {"ms": round(ms, 4), "edges_per_s": round(Es / (ms * 1e-3), 1),
                    "algorithmic_GBs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
        log(f"shard {k:10s} {ms * 1e3:8.1f} us  {gbs:8.1f} GB/s algorithmic "
            f"({100 * gbs / HBM_PEAK_GBS:.1f} % of 8 TB/s)")
    log(f"shard: {sh.n_owned} owned + {sh.n_halo} halo nodes, {Es} edges; owned residual vs "
        f"the whole mesh {err:.2e}")
    out = {"split": "2x2x2 blocks of the box; the central block", "owned_nodes": sh.n_owned,
           "halo_nodes": sh.n_halo, "edges": Es, "forms": forms,
           "owned_residual_error_vs_whole_mesh": float(f"{err:.3e}")}
    del ps, ps32
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--variant", default="owner",
                    choices=["owner", "coloured", "atomic", "coloured-lds-atomic", "flat"])
    ap.add_argument("--cluster-size", type=int, default=512)
    ap.add_argument("--no-lane-groups", action="store_true")
    ap.add_argument("--no-bank-spread", action="store_true")
    ap.add_argument("--no-halo-order", action="store_true")
    ap.add_argument("--renumber", choices=["rcm", "morton", "none"], default="morton")
    ap.add_argument("--block-size", type=int, default=512)
    ap.add_argument("--colour-sort", action="store_true")
    ap.add_argument("--mesh", choices=sorted(MESHES), default="E",
                    help="E: 160^3 layered 5/6-tet box (4.1M nodes); B: 100^3 6-tet box (1M nodes); "
                         "A: 20^3 6-tet box (8,000 nodes)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one 1 GiB device copy first (calibrates profiler byte counters)")
    ap.add_argument("--cpu-baseline-only", action="store_true",
                    help="time the oracle on the host (three meshes) and print that JSON line")
    args = ap.parse_args()
    if args.cpu_baseline_only:
        print(json.dumps(cpu_baseline_sweep()), flush=True)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (it would "
              "shard by owned node partitions, each GPU importing its halo's state once per "
              "stage)", file=sys.stderr)
        sys.exit(2)

    import torch

    import meshgen
    import paper_1403_7209_amd as pk

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    variant = pk.VARIANTS[args.variant]

    t0 = time.perf_counter()
    mn, msplit, mjit, mdesc = MESHES[args.mesh]
    mesh = meshgen.build_mesh(mn, msplit, mjit)
    q = meshgen.state(mesh.N, mesh.perm)
    N, E = mesh.N, mesh.E
    log(f"mesh: N={N} E={E} ({time.perf_counter() - t0:.1f} s)")

    ctx = pk.Context(dev)
    t0 = time.perf_counter()
    t2n = mesh.tets()
    t2e = meshgen.tet_edges(mesh, t2n)
    p64 = pk.FluxProblem(ctx, mesh.e2n, mesh.w, mesh.vol, q, renumber=args.renumber,
                         block_size=args.block_size, colour_sort=args.colour_sort,
                         coords=mesh.xyz, cluster_size=args.cluster_size,
                         lane_groups=not args.no_lane_groups, tets=t2n, tet_edges=t2e,
                         bank_spread=not args.no_bank_spread, halo_order=not args.no_halo_order)
    T = len(t2n)
    p32 = pk.FluxProblem(ctx, mesh.e2n, mesh.w, mesh.vol, q, fp32=True, like=p64)
    info = p64.info
    log(f"plan: {info['plan_seconds']:.1f} s, nb={info['nblocks']} nc={info['nblock_colours']} "
        f"sumU/N={info['sum_unique'] / N:.3f} maxU={info['max_unique']} "
        f"edge colours mean {info['mean_elem_colours']:.1f} ({time.perf_counter() - t0:.1f} s)")

    dt = p64.compute_dt(0.5, variant)
    rbar = torch.from_numpy(meshgen.normal(6 * N, purpose=21).reshape(6, N)).to(dev)
    qbar = torch.zeros((6, N), dtype=torch.float64, device=dev)
    nbar = torch.empty((3, E), dtype=torch.float64, device=dev)
    rbar_d, qbar_d = p64.dat(rbar, "rbar"), p64.dat(qbar, "qbar")
    nbar_d = p64.dat(nbar, "nbar", edges=True)
    q0_init64, q0_init32 = p64.qa.clone(), p32.qa.clone()

    stream = torch.cuda.current_stream(dev)
    timers = {k: [] for k in ("fp64", "fp32", "adjoint", "rk64", "rk32", "fp64_fused",
                              "fp32_fused")}
    if args.copy_probe:
        src = torch.ones(2 ** 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def ev():
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        return e

    # the owner variant writes each residual once, so the stage need not zero it
    ra, rk = (pk.WRITE, pk.READ) if variant == pk.OWNER else (pk.INC, pk.RW)

    fused = variant == pk.OWNER
    for p in (p64, p32):
        p.qc = torch.empty_like(p.qa)

    def rk_iter(p, kflux, krk, rec):
        qa, qb = p.dat(p.qa, "qa"), p.dat(p.qb, "qb")
        p.ss.zero_()
        if fused:  # stage k reads stage k-1's state and writes the other buffer
            bufs = (qb, p.dat(p.qc, "qc"))
            src = qa
            for k in range(5):
                a = ev() if rec else None
                p.ctx.edge_flux_stage(p.edges, p.e2n, src, p.w, qa, p.vol, bufs[k % 2],
                                      pk.RK_ALPHA[k] * dt, p.ss[k], p.gamma)
                b = ev() if rec else None
                if rec:
                    timers[kflux + "_fused"].append((a, b))
                src = bufs[k % 2]
            p.qa, p.qb = p.qb, p.qa
            return
        for k in range(5):
            a = ev() if rec else None
            p.ctx.edge_flux(p.edges, p.e2n, qa if k == 0 else qb, p.w, p.res_d, p.gamma, variant,
                            ra)
            b = ev() if rec else None
            p.ctx.rk_stage(p.nodes, qa, p.res_d, p.vol, qb, pk.RK_ALPHA[k] * dt, p.ss[k],
                           rk)
            c = ev() if rec else None
            if rec:
                timers[kflux].append((a, b))
                timers[krk].append((b, c))
        p.qa, p.qb = p.qb, p.qa

    def step(rec):
        rk_iter(p64, "fp64", "rk64", rec)
        rk_iter(p32, "fp32", "rk32", rec)
        if variant != pk.OWNER:
            qbar.zero_()
        a = ev() if rec else None
        ctx.edge_flux_adjoint(p64.edges, p64.e2n, p64.dat(p64.qa, "q"), p64.w, rbar_d, qbar_d,
                              nbar_d, p64.gamma, variant, ra)
        b = ev() if rec else None
        if rec:
            timers["adjoint"].append((a, b))

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    # restart from the initial state so every run times the same iterations
    p64.qa.copy_(q0_init64)
    p32.qa.copy_(q0_init32)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    e_start = ev()
    for _ in range(args.steps):
        step(True)
    e_end = ev()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    ms_step = e_start.elapsed_time(e_end) / args.steps
    ctx.sync()
    if not ctx.check_finite(p64.ss) or not ctx.check_finite(p32.ss):
        log("warning: non-finite residual norm")
    # both forms ran the same iterations from the same state: the FP32-storage
    # form's error, per variable relative to the FP64 state's largest value
    a64, a32 = p64.qa.double(), p32.qa.double()
    err32 = float(((a64 - a32).abs().amax(dim=1) / a64.abs().amax(dim=1)).max())
    log(f"FP32-storage state vs FP64 after {args.steps} iterations: {err32:.2e}")

    # the plain edge loops (residual written), beside the step when it fuses the stage
    if fused:
        for rec in (False, True):
            for _ in range(3 if rec else 1):
                for p, key in ((p64, "fp64"), (p32, "fp32")):
                    a = ev()
                    p.ctx.edge_flux(p.edges, p.e2n, p.dat(p.qa, "qa"), p.w, p.res_d, p.gamma,
                                    variant, pk.WRITE)
                    b = ev()
                    if rec:
                        timers[key].append((a, b))

    # loops beside the step: Green-Gauss gradient, second-order flux, local dt
    p64.set_edge_vectors(meshgen.edge_vectors(mesh))
    G = torch.empty((18, N), dtype=torch.float64, device=dev)
    res2 = torch.empty((6, N), dtype=torch.float64, device=dev)
    ga = pk.WRITE if variant == pk.OWNER else pk.INC
    second_order = True
    try:  # the 24-value records of these loops may not fit a plan's partitions in LDS
        p64.gradient(p64.qa, G, variant, ga)
        p64.residual2(p64.qa, G, res2, variant, ga)
    except pk.OpfError as err:
        log(f"gradient and second-order loops not run with this plan: {err}")
        second_order = False
    for rec in (False, True):
        for _ in range(3 if rec else 1):
            if ga == pk.INC:
                G.zero_()
                res2.zero_()
            a = ev()
            if second_order:
                p64.gradient(p64.qa, G, variant, ga)
            b = ev()
            if second_order:
                p64.residual2(p64.qa, G, res2, variant, ga)
            c = ev()
            p64.compute_local_dt(0.5, variant)
            d = ev()
            if rec and second_order:
                timers.setdefault("grad", []).append((a, b))
                timers.setdefault("flux2", []).append((b, c))
            p64.ctx.local_dt(p64.nodes, p64.vol, p64.lam_d, 0.5, p64.dtl_d)
            e = ev()
            if rec:
                timers.setdefault("local_dt", []).append((d, e))
    # the geometry loop over the tets and its reverse
    x = p64.nodes_in(mesh.xyz)
    wg = torch.empty((3, E), dtype=torch.float64, device=dev)
    volg = torch.empty(N, dtype=torch.float64, device=dev)
    xbar = torch.empty((3, N), dtype=torch.float64, device=dev)
    for rec in (False, True):
        for _ in range(3 if rec else 1):
            for variant, tag in ((pk.OWNER, ""), (pk.ATOMIC, "_atomic")):
                # the gather form writes its results; the scatter form adds into zeros
                if variant == pk.ATOMIC:
                    wg.zero_()
                    volg.zero_()
                xbar.zero_()
                a = ev()
                p64.geometry(x, wg, volg, variant=variant,
                             access=pk.WRITE if variant == pk.OWNER else pk.INC)
                b = ev()
                p64.geometry_adjoint(x, nbar, volg, xbar, variant=variant)
                c = ev()
                if rec:
                    timers.setdefault("geometry" + tag, []).append((a, b))
                    timers.setdefault("geometry_adj" + tag, []).append((b, c))
    torch.cuda.synchronize()

    # one GPU's share of the mesh split over eight (owned block, halo, every edge
    # with an owned end), against the whole mesh's residual of the same state
    shard = None
    if fused and N >= 8 * 512:
        res_full = torch.empty((6, N), dtype=torch.float64, device=dev)
        ctx.edge_flux(p64.edges, p64.e2n, p64.dat(q0_init64, "q0"), p64.w,
                      p64.dat(res_full, "rfull"), p64.gamma, pk.OWNER, pk.WRITE)
        torch.cuda.synchronize()
        res_user = p64.nodes_out(res_full)
        del res_full
        shard = shard_share(pk, ctx, mesh, q, mn, dt, rbar_user=meshgen.normal(6 * N, purpose=21)
                            .reshape(6, N), res_user=res_user, ev=ev)
        del res_user

    # a device-to-device copy of 1 GiB for context: what plain streaming reaches here
    src = torch.ones(2 ** 27, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    a = ev()
    for _ in range(5):
        dst.copy_(src)
    b = ev()
    torch.cuda.synchronize()
    copy_gbs = 5 * 2 * src.numel() * 8 / (a.elapsed_time(b) * 1e-3) / 1e9
    del src, dst
    log(f"device copy {copy_gbs:.1f} GB/s (read + write)")

    per = {}
    for k, lst in timers.items():
        if not lst:
            continue
        times = [a.elapsed_time(b) for a, b in lst]
        ms = float(np.mean(times))
        be, bn, bt = (*BYTES[k], 0)[:3]
        gbs = (be * E + bn * N + bt * T) / (ms * 1e-3) / 1e9
        per[k] = {"ms": round(ms, 4), "ms_median": round(float(np.median(times)), 4),
                  "ms_min": round(float(np.min(times)), 4), "launches": len(times),
                  "algorithmic_GBs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                  "frac_of_device_copy": round(gbs / copy_gbs, 4)}
        if be:
            per[k]["edges_per_s"] = round(E / (ms * 1e-3), 1)
        log(f"{k:8s} {ms * 1e3:9.1f} us  {gbs:8.1f} GB/s algorithmic  "
            f"({100 * gbs / HBM_PEAK_GBS:.1f} % of 8 TB/s, "
            f"{100 * gbs / copy_gbs:.1f} % of the device copy)")
    main64, main32 = ("fp64_fused", "fp32_fused") if fused else ("fp64", "fp32")
    speedup32 = per[main64]["ms"] / per[main32]["ms"]
    value = 11 * E / (ms_step * 1e-3)
    log(f"step {ms_step:.3f} ms (wall {1e3 * wall / args.steps:.3f} ms), {value:.4e} edges/s, "
        f"FP32/FP64 loop speedup {speedup32:.3f}")

    dom = per[main64]
    be, bn = BYTES[main64]
    config_key = (f"n={mn} variant={args.variant} renumber={args.renumber} "
                  f"cluster={args.cluster_size} block={args.block_size} "
                  f"lane_groups={not args.no_lane_groups} colour_sort={bool(args.colour_sort)} "
                  f"bank_spread={not args.no_bank_spread} halo_order={not args.no_halo_order}")
    out = {
        "metric": "edges/s of edge-flux residual loop (FP64, FP32, adjoint) + % HBM roofline",
        "value": round(value, 1),
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"periodic {mn}^3 box, {mdesc}, jitter {mjit}h: "
                        f"N={N} nodes, E={E} edges; step = FP64 RK5 iteration + FP32-storage "
                        f"RK5 iteration + 1 FP64 adjoint sweep (11 edge loops)",
            "variant": args.variant,
            "renumber": args.renumber,
            "block_size": args.block_size,
            "colour_sort": bool(args.colour_sort),
            "cluster_size": args.cluster_size,
            "lane_groups": not args.no_lane_groups,
            "bank_spread": not args.no_bank_spread,
            "halo_order": not args.no_halo_order,
            "plan": {k: info[k] for k in ("nblocks", "nblock_colours", "sum_unique", "max_unique",
                                          "mean_elem_colours", "nclusters", "owner_edge_visits",
                                          "plan_seconds")},
        },
        "forms": per,
        "fp32_speedup_over_fp64": round(speedup32, 4),
        "fp32_error_vs_fp64": float(f"{err32:.3e}"),
        "shard_of_8": shard,
        "roofline": {
            "kernel": ("FP64 edge-flux loop with the stage update fused (opf_edge_flux_stage)"
                       if fused else "FP64 edge-flux loop (opf_edge_flux)"),
            "bound": "hbm",
            "achieved": dom["algorithmic_GBs"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": dom["hbm_frac"],
            "bytes_per_launch": be * E + bn * N,
            "traffic": measured_traffic(config_key),
            "device_copy_GBs": round(copy_gbs, 1),
            "frac_of_device_copy": dom["frac_of_device_copy"],
        },
    }
    if not args.no_cpu_baseline:
        log("timing the oracle on the host ...")
        # the residual of the initial state from both forms (the FP32-storage
        # form from the state rounded to FP32, as it stores it), for the
        # oracle leg to compare with its own
        gpu_res = {}
        for tag, p, q0 in (("fp64", p64, q0_init64), ("fp32", p32, q0_init32)):
            r = torch.zeros((6, N), dtype=torch.float64, device=dev)
            own = bool(p.info["owner_ok"])
            p.residual(q0, r, pk.OWNER if own else pk.ATOMIC, pk.WRITE if own else pk.INC)
            torch.cuda.synchronize()
            gpu_res[tag] = p.nodes_out(r)
        out["cpu_baseline"] = cpu_baseline(mesh, q, gpu_res)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
