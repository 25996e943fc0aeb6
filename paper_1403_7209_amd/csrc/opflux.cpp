// opflux.cpp -- C ABI of libopflux: context, declarations, plans and loops.
//
// Follows the OP2 model (Sec. 3.1-3.2): sets, maps and dats are declared once;
// the library owns the maps and may renumber the sets; an op_par_loop-style
// call names a kernel and describes each argument (dat, map column, map,
// dimension, type, access), and the library checks that description against
// the kernel's fixed signature before launching it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <initializer_list>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "kernels.hpp"
#include "opflux.h"
#include "planner.hpp"

namespace {

struct SetRec {
    int64_t size = 0;
    std::string name;
    int plan_map = -1;  // map whose plan renumbered this set
};

struct MapRec {
    opf_set from = -1, to = -1;
    int dim = 0;
    std::vector<int32_t> idx;  // 0-based, row-major
    std::string name;
    uint64_t version = 0;
};

struct DatRec {
    opf_set set = -1;
    int dim = 0;
    int type = 0;
    void *ptr = nullptr;
    int64_t ld = 0;
    std::string name;
};

struct PlanRec {
    opf::Plan host;
    opf::gpu::DevPlan dev;
    std::vector<void *> bufs;
    uint64_t map_version = 0;
    int64_t device_bytes = 0;
    bool on_device = false;
};

size_t type_size(int t) { return t == OPF_F32 ? 4 : 8; }

}  // namespace

// Device copy of a map in internal numbering (tet loops), keyed by map.
struct DevMap {
    uint64_t version = 0;
    int32_t *ptr = nullptr;
};

// Incident tets of every edge and node (gather form of the tet loops), keyed
// by the (t2n, t2e) pair.
struct DevTetInverse {
    uint64_t vn = 0, ve = 0;
    int32_t *t2n = nullptr, *t2e = nullptr;  // tets in the gather order
    int32_t *e2t_off = nullptr, *e2t = nullptr, *n2t_off = nullptr, *n2t = nullptr;
    int32_t *n2t_pos = nullptr;
    double *scratch = nullptr;  // kTetScratch values per tet
    double *wT = nullptr;       // the reverse's interleaved copy of wbar
    // ring form of the forward (see opf::gpu::TetArrays); ring == nullptr when
    // the mesh does not fit it
    int32_t *ring_off = nullptr, *chunk_e = nullptr, *halo_off = nullptr, *halo = nullptr;
    int32_t *vsec_off = nullptr, *vsec = nullptr, *vloc_off = nullptr;
    uint16_t *ring = nullptr, *vloc = nullptr;
    double *edge_det = nullptr;
    int nchunk = 0, KG = 0, L = 0, RB = 0, DV = 0;
};

struct opf_ctx {
    int device = -1;
    std::string err;
    std::vector<SetRec> sets;
    std::vector<MapRec> maps;
    std::vector<DatRec> dats;
    std::map<int, std::unique_ptr<PlanRec>> plans;
    std::map<int, DevMap> dmaps;
    std::map<std::pair<int, int>, DevTetInverse> tinv;
    void *(*alloc_fn)(void *, size_t) = nullptr;
    void (*free_fn)(void *, void *) = nullptr;
    void *alloc_user = nullptr;
    double *scratch = nullptr;  // partial sums of the direct reductions
    // Library-owned scratch (the reductions' partial sums, the fused stage's
    // per-cluster partials, the tet records of the gather form) is shared by
    // every call on this context.  After each call that uses it, an event is
    // recorded on that call's stream; a call on another stream first waits for
    // it, so calls on different streams never overlap on the scratch.
    hipEvent_t scratch_ev = nullptr;
    hipStream_t scratch_stream = nullptr;
    bool scratch_used = false;
    size_t max_lds = 65536;
    size_t lds_limit = 65536;
    uint64_t next_version = 1;

    int fail(int code, const std::string &msg)
    {
        err = msg;
        return code;
    }
    void *dalloc(size_t bytes)
    {
        if (bytes == 0) bytes = 256;
        if (alloc_fn) {
            void *p = alloc_fn(alloc_user, bytes);
            if (p && (reinterpret_cast<uintptr_t>(p) & 15u)) {  // the kernels need 16-byte words
                if (free_fn) free_fn(alloc_user, p);
                return nullptr;
            }
            return p;
        }
        void *p = nullptr;
        return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
    }
    void dfree(void *p)
    {
        if (!p) return;
        if (free_fn)
            free_fn(alloc_user, p);
        else
            (void)hipFree(p);
    }
    bool set_ok(opf_set s) const { return s >= 0 && s < (opf_set)sets.size(); }
    bool map_ok(opf_map m) const { return m >= 0 && m < (opf_map)maps.size(); }
    bool dat_ok(opf_dat d) const { return d >= 0 && d < (opf_dat)dats.size(); }
};

namespace {

int hip_fail(opf_ctx *ctx, hipError_t e, const char *what)
{
    return ctx->fail(OPF_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

void free_plan(opf_ctx *ctx, PlanRec &p)
{
    for (void *b : p.bufs) ctx->dfree(b);
    p.bufs.clear();
    p.on_device = false;
}

template <typename T>
int upload(opf_ctx *ctx, PlanRec &p, const std::vector<T> &v, const T *&out)
{
    const size_t bytes = v.size() * sizeof(T);
    void *d = ctx->dalloc(bytes);
    if (!d) return ctx->fail(OPF_ENOMEM, "device allocation of plan arrays failed");
    p.bufs.push_back(d);
    p.device_bytes += (int64_t)bytes;
    if (bytes) {
        hipError_t e = hipMemcpy(d, v.data(), bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(ctx, e, "plan upload");
    }
    out = static_cast<const T *>(d);
    return OPF_OK;
}

// The owner kernel's arrays (see DevPlan): per cluster the interior block and
// the cut visits; per interior edge a word of the two ends' offsets in the
// cluster and the bank-spreading flag.
int upload_owner(opf_ctx *ctx, PlanRec &pr)
{
    const opf::Plan &P = pr.host;
    opf::gpu::DevPlan &D = pr.dev;
    const int K = P.cluster_size;
    const int64_t ncl = P.nclusters();
    std::vector<int2> iblk(ncl);
    std::vector<uint32_t> iw(P.E, 0);
    for (int64_t c = 0; c < ncl; ++c) {
        const int32_t p0 = P.cl_prim[2 * c], ni = P.cl_nint[c];
        iblk[c] = make_int2(p0, ni);
        for (int64_t e = p0; e < p0 + ni; ++e) {
            const uint32_t sw = P.owner_swap.empty() ? 0u : (uint32_t)P.owner_swap[e];
            iw[e] = (uint32_t)(P.e2n[2 * e] - c * K) | ((uint32_t)(P.e2n[2 * e + 1] - c * K) << 16) |
                    (sw << 31);
        }
    }
    const size_t nv = P.cl_cut_eid.size();
    std::vector<int> cv_off(ncl + 1);
    for (int64_t c = 0; c <= ncl; ++c) cv_off[c] = (int)P.cl_cut_off[c];
    int rc = upload(ctx, pr, iblk, D.iblk);
    if (!rc) rc = upload(ctx, pr, iw, D.iw);
    if (!rc) rc = upload(ctx, pr, cv_off, D.cv_off);
    // both orders of the cut visits: edge, other end | orientation, owned offset
    for (int order = 0; order < 2 && !rc; ++order) {
        const std::vector<int32_t> &ce = order ? P.cl_cutf_eid : P.cl_cut_eid;
        const std::vector<uint8_t> &ch = order ? P.cl_cutf_end : P.cl_cut_end;
        std::vector<int> cv_oth(nv);
        std::vector<uint16_t> cv_own(nv);
        for (int64_t c = 0; c < ncl; ++c)
            for (int64_t s = P.cl_cut_off[c]; s < P.cl_cut_off[c + 1]; ++s) {
                const int64_t e = ce[s];
                const int h = ch[s];
                cv_oth[s] = (int)((uint32_t)P.e2n[2 * e + 1 - h] | ((uint32_t)h << 31));
                cv_own[s] = (uint16_t)(P.e2n[2 * e + h] - c * K);
            }
        rc = upload(ctx, pr, ce, order ? D.cvf_eid : D.cv_eid);
        if (!rc) rc = upload(ctx, pr, cv_oth, order ? D.cvf_oth : D.cv_oth);
        if (!rc) rc = upload(ctx, pr, cv_own, order ? D.cvf_own : D.cv_own);
    }
    return rc;
}

int upload_plan(opf_ctx *ctx, PlanRec &pr)
{
    const opf::Plan &P = pr.host;
    if (P.E >= (int64_t)1 << 31 || (int64_t)P.uniq.size() >= (int64_t)1 << 31)
        return ctx->fail(OPF_ESIZE, "plan too large for 32-bit device offsets");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
    const int64_t nb = P.nblocks();
    std::vector<int2> e2n(P.E);
    for (int64_t k = 0; k < P.E; ++k) e2n[k] = make_int2(P.e2n[2 * k], P.e2n[2 * k + 1]);
    std::vector<int> block_off(nb + 1), uniq_off(nb + 1);
    for (int64_t b = 0; b <= nb; ++b) {
        block_off[b] = (int)P.block_off[b];
        uniq_off[b] = (int)P.uniq_off[b];
    }
    std::vector<uint32_t> lidx(P.E);
    for (int64_t k = 0; k < P.E; ++k)
        lidx[k] = (uint32_t)P.lidx[2 * k] | ((uint32_t)P.lidx[2 * k + 1] << 16);
    opf::gpu::DevPlan &D = pr.dev;
    D = opf::gpu::DevPlan();
    D.N = (int)P.N;
    D.E = (int)P.E;
    D.nb = (int)nb;
    D.nc = P.nblock_colours;
    D.umax = P.max_unique;
    D.block_size = P.block_size;
    D.colour_off.assign(P.colour_off.begin(), P.colour_off.end());
    int rc = OPF_OK;
    D.K = P.cluster_size;
    D.ncl = (int)P.nclusters();
    D.owner_ok = P.owner_ok && D.ncl > 0;
    if (D.owner_ok) {
        if (P.cluster_size > 8192) return ctx->fail(OPF_EINVAL, "cluster_size above 8192");
        rc = upload_owner(ctx, pr);
        if (!rc) {
            const size_t nb = sizeof(double) * (opf::gpu::kSumTail + 6 * (size_t)D.ncl);
            D.stage_partial = static_cast<double *>(ctx->dalloc(nb));
            if (!D.stage_partial) {
                rc = ctx->fail(OPF_ENOMEM, "device allocation of plan arrays failed");
            } else {
                pr.bufs.push_back(D.stage_partial);
                // the second pass's counter starts at zero
                const hipError_t e = hipMemset(D.stage_partial, 0, nb);
                if (e != hipSuccess) rc = hip_fail(ctx, e, "clearing the stage partial sums");
            }
        }
    }
    if (P.flat_ok) {
        D.nflat = P.flat_colours;
        D.flat_off.assign(P.flat_off.begin(), P.flat_off.end());
        if (!rc) rc = upload(ctx, pr, P.flat_eid, D.flat_eid);
    }
    if (!rc) rc = upload(ctx, pr, e2n, D.e2n);
    if (P.coloured_ok) {
        if (!rc) rc = upload(ctx, pr, block_off, D.block_off);
        if (!rc) rc = upload(ctx, pr, uniq_off, D.uniq_off);
        if (!rc) rc = upload(ctx, pr, P.uniq, D.uniq);
        if (!rc) rc = upload(ctx, pr, lidx, D.lidx);
        if (!rc) rc = upload(ctx, pr, P.ecol, D.ecol);
        if (!rc) rc = upload(ctx, pr, P.block_ncol, D.block_ncol);
        if (!rc) rc = upload(ctx, pr, P.colour_blocks, D.colour_blocks);
    } else {
        D.nc = 0;
        D.colour_off.assign(1, 0);
    }
    if (rc) {
        free_plan(ctx, pr);
        return rc;
    }
    pr.on_device = true;
    return OPF_OK;
}

// Expected shape of one loop argument.
struct Want {
    opf_set set;  // set the dat lives on
    int idx;      // map column, or -1
    opf_map map;  // map, or OPF_ID
    int dim;
    int type;     // -1: any of F64/F32 (checked by the caller)
    int access;
};

int check_arg(opf_ctx *ctx, const opf_arg &a, const Want &w, int pos)
{
    const std::string at = "argument " + std::to_string(pos) + ": ";
    if (!ctx->dat_ok(a.dat)) return ctx->fail(OPF_EINVAL, at + "invalid dat handle");
    const DatRec &d = ctx->dats[a.dat];
    if (a.map != w.map || a.idx != w.idx)
        return ctx->fail(OPF_EINVAL, at + "expected map " + std::to_string(w.map) + " index " +
                                         std::to_string(w.idx));
    if (d.set != w.set) return ctx->fail(OPF_EINVAL, at + "dat '" + d.name + "' is on the wrong set");
    if (a.dim != w.dim || d.dim != w.dim)
        return ctx->fail(OPF_ESIZE, at + "expected dimension " + std::to_string(w.dim));
    if (a.type != d.type) return ctx->fail(OPF_ETYPE, at + "type differs from the dat's type");
    if (w.type >= 0 && a.type != w.type) return ctx->fail(OPF_ETYPE, at + "wrong data type");
    if (a.access != w.access) return ctx->fail(OPF_EACCESS, at + "wrong access mode");
    return OPF_OK;
}

int check_gbl(opf_ctx *ctx, const opf_gbl &g, int dim, int access, int on_device, int pos)
{
    const std::string at = "global " + std::to_string(pos) + ": ";
    if (!g.ptr) return ctx->fail(OPF_EINVAL, at + "NULL pointer");
    if (g.dim != dim) return ctx->fail(OPF_ESIZE, at + "expected dimension " + std::to_string(dim));
    if (g.type != OPF_F64) return ctx->fail(OPF_ETYPE, at + "globals are F64");
    if (g.access != access) return ctx->fail(OPF_EACCESS, at + "wrong access mode");
    if (g.on_device != on_device)
        return ctx->fail(OPF_EINVAL, at + (on_device ? "must be device memory" : "must be host memory"));
    return OPF_OK;
}

const void *comp(const DatRec &d, int c)
{
    return static_cast<const char *>(d.ptr) + (size_t)c * (size_t)d.ld * type_size(d.type);
}

// Makes the context's device current; allocates nothing.
int device_bind(opf_ctx *ctx)
{
    if (ctx->device < 0) return ctx->fail(OPF_EDEVICE, "host-only context cannot run loops");
    const hipError_t e = hipSetDevice(ctx->device);
    return e == hipSuccess ? OPF_OK : hip_fail(ctx, e, "hipSetDevice");
}

// Device address of the static scratch (the allocation-free fused loop), per
// device, resolved by opf_init with that device current.
constexpr int kMaxStaticDevices = 64;
std::mutex g_static_mu;
double *g_static_scratch[kMaxStaticDevices] = {};

double *static_scratch_of(int device)
{
    if (device < 0 || device >= kMaxStaticDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_static_mu);
    return g_static_scratch[device];
}

// Resolves the static scratch of `device` once; restores the caller's device.
int resolve_static_scratch(int device)
{
    if (device >= kMaxStaticDevices) return OPF_OK;  // the allocation-free loop then refuses
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (g_static_scratch[device]) return OPF_OK;
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (hipSetDevice(device) != hipSuccess) return OPF_EDEVICE;
    double *p = nullptr;
    const int e = opf::gpu::static_scratch_address(&p);
    if (prev >= 0) (void)hipSetDevice(prev);
    if (e || !p) return OPF_EDEVICE;
    g_static_scratch[device] = p;
    return OPF_OK;
}

int device_ready(opf_ctx *ctx)
{
    if (ctx->device < 0) return ctx->fail(OPF_EDEVICE, "host-only context cannot run loops");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
    if (!ctx->scratch) {
        const size_t nb = sizeof(double) * (opf::gpu::kSumTail + 6 * opf::gpu::kRkBlocks);
        ctx->scratch = static_cast<double *>(ctx->dalloc(nb));
        if (!ctx->scratch) return ctx->fail(OPF_ENOMEM, "scratch allocation failed");
        const hipError_t e = hipMemset(ctx->scratch, 0, nb);  // the second pass's counter
        if (e != hipSuccess) return hip_fail(ctx, e, "clearing the scratch");
    }
    return OPF_OK;
}

// Orders a call that uses library-owned scratch on stream `st` after the last
// such call, whatever stream that ran on.
int scratch_begin(opf_ctx *ctx, hipStream_t st)
{
    if (!ctx->scratch_ev) {
        hipError_t e = hipEventCreateWithFlags(&ctx->scratch_ev, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(ctx, e, "scratch event");
    }
    if (ctx->scratch_used && st != ctx->scratch_stream) {
        hipError_t e = hipStreamWaitEvent(st, ctx->scratch_ev, 0);
        if (e != hipSuccess) return hip_fail(ctx, e, "waiting for the previous stream's scratch use");
    }
    return OPF_OK;
}

int scratch_end(opf_ctx *ctx, hipStream_t st)
{
    hipError_t e = hipEventRecord(ctx->scratch_ev, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "recording the scratch event");
    ctx->scratch_used = true;
    ctx->scratch_stream = st;
    return OPF_OK;
}

// Byte range [lo, hi) spanned by a dat's elements (its last component ends at
// (dim - 1) * ld + size); empty for a NULL pointer (host-only contexts).
struct ByteRange {
    uintptr_t lo = 0, hi = 0;
};

ByteRange dat_range(const opf_ctx *ctx, opf_dat d)
{
    ByteRange r;
    const DatRec &dr = ctx->dats[d];
    if (!dr.ptr) return r;
    const int64_t n = ctx->sets[dr.set].size;
    r.lo = reinterpret_cast<uintptr_t>(dr.ptr);
    r.hi = r.lo + (uintptr_t)(((int64_t)(dr.dim - 1) * dr.ld + n) * (int64_t)type_size(dr.type));
    return r;
}

bool overlap(ByteRange a, ByteRange b) { return a.lo < a.hi && b.lo < b.hi && a.lo < b.hi && b.lo < a.hi; }

// An output (WRITE, RW or INC) must share no byte with another argument: the
// kernels read inputs and write outputs from different workgroups in no fixed
// order.  Dats are compared by the memory they cover, not by handle, so two
// handles declared over one buffer are caught too.
int check_disjoint(opf_ctx *ctx, opf_dat out, std::initializer_list<opf_dat> others, const char *what)
{
    const ByteRange ro = dat_range(ctx, out);
    for (opf_dat o : others) {
        if (o < 0) continue;  // an optional argument left out
        if (o == out) return ctx->fail(OPF_EINVAL, std::string(what) + ": output aliases an input");
        if (overlap(ro, dat_range(ctx, o)))
            return ctx->fail(OPF_EINVAL, std::string(what) + ": output '" + ctx->dats[out].name +
                                             "' overlaps the memory of '" + ctx->dats[o].name + "'");
    }
    return OPF_OK;
}

// The same for a device global (6 or 1 doubles) against the dats of a loop.
int check_gbl_disjoint(opf_ctx *ctx, const void *p, size_t bytes, std::initializer_list<opf_dat> dats,
                       const char *what)
{
    ByteRange g;
    g.lo = reinterpret_cast<uintptr_t>(p);
    g.hi = g.lo + bytes;
    for (opf_dat d : dats)
        if (d >= 0 && overlap(g, dat_range(ctx, d)))
            return ctx->fail(OPF_EINVAL, std::string(what) + ": the device global overlaps '" +
                                             ctx->dats[d].name + "'");
    return OPF_OK;
}

int edge_loop(opf_ctx *ctx, int kernel, opf_set s, int nargs, const opf_arg *args, int ngbl,
              const opf_gbl *gbls, int variant, hipStream_t st)
{
    const bool adj = kernel == OPF_K_EDGE_FLUX_ADJ, grad = kernel == OPF_K_EDGE_GRAD,
               flux2 = kernel == OPF_K_EDGE_FLUX2;
    const int want_args = adj ? 8 : flux2 ? 10 : 5;
    if (nargs != want_args || !args)
        return ctx->fail(OPF_EINVAL, "expected " + std::to_string(want_args) + " arguments");
    const int want_gbl = grad ? 0 : 1;
    if (ngbl != want_gbl || (want_gbl && !gbls))
        return ctx->fail(OPF_EINVAL, grad ? "expected no globals" : "expected one global (gamma)");
    if (variant < OPF_V_COLOURED || variant > OPF_V_FLAT)
        return ctx->fail(OPF_EINVAL, "unknown variant");
    const opf_map m = args[0].map;
    if (!ctx->map_ok(m)) return ctx->fail(OPF_EINVAL, "argument 0: invalid map");
    const MapRec &mr = ctx->maps[m];
    if (mr.dim != 2 || mr.from != s)
        return ctx->fail(OPF_EINVAL, "the loop set must be the source set of an arity-2 map");
    if (!ctx->dat_ok(args[0].dat)) return ctx->fail(OPF_EINVAL, "argument 0: invalid dat");
    const int T = ctx->dats[args[0].dat].type;
    if (T != OPF_F64 && T != OPF_F32) return ctx->fail(OPF_ETYPE, "argument 0: unknown type");
    if ((adj || grad || flux2) && T != OPF_F64)
        return ctx->fail(OPF_ETYPE, "the adjoint, gradient and second-order loops are FP64 only");
    const opf_set nodes = mr.to;
    int rc = OPF_OK;
    // expected signature; `yslot` is the first of the two node-increment arguments
    std::vector<Want> w = {{nodes, 0, m, 6, T, OPF_READ}, {nodes, 1, m, 6, T, OPF_READ}};
    int yslot = 3;
    if (adj) {
        w.push_back({s, -1, OPF_ID, 3, T, OPF_READ});
        w.push_back({nodes, 0, m, 6, OPF_F64, OPF_READ});
        w.push_back({nodes, 1, m, 6, OPF_F64, OPF_READ});
        w.push_back({nodes, 0, m, 6, OPF_F64, OPF_INC});
        w.push_back({nodes, 1, m, 6, OPF_F64, OPF_INC});
        w.push_back({s, -1, OPF_ID, 3, OPF_F64, OPF_WRITE});
        yslot = 5;
    } else if (flux2) {
        w.push_back({nodes, 0, m, 18, OPF_F64, OPF_READ});
        w.push_back({nodes, 1, m, 18, OPF_F64, OPF_READ});
        w.push_back({nodes, 0, m, 1, OPF_F64, OPF_READ});
        w.push_back({nodes, 1, m, 1, OPF_F64, OPF_READ});
        w.push_back({s, -1, OPF_ID, 3, OPF_F64, OPF_READ});
        w.push_back({s, -1, OPF_ID, 3, OPF_F64, OPF_READ});
        w.push_back({nodes, 0, m, 6, OPF_F64, OPF_INC});
        w.push_back({nodes, 1, m, 6, OPF_F64, OPF_INC});
        yslot = 8;
    } else {
        const int yd = kernel == OPF_K_EDGE_SPECRAD ? 1 : grad ? 18 : 6;
        w.push_back({s, -1, OPF_ID, 3, T, OPF_READ});
        w.push_back({nodes, 0, m, yd, OPF_F64, OPF_INC});
        w.push_back({nodes, 1, m, yd, OPF_F64, OPF_INC});
    }
    // The owner variant writes every node's total exactly once, so it also
    // accepts WRITE on the node increments (res = sum, no prior zeroing).
    bool overwrite = false;
    if (variant == OPF_V_OWNER && args[yslot].access == OPF_WRITE &&
        args[yslot + 1].access == OPF_WRITE) {
        w[yslot].access = w[yslot + 1].access = OPF_WRITE;
        overwrite = true;
    }
    for (int k = 0; k < nargs && !rc; ++k) rc = check_arg(ctx, args[k], w[k], k);
    if (rc) return rc;
    // the two map columns of a node argument must name the same dat
    auto same = [&](int a, int b) {
        return args[a].dat == args[b].dat
                   ? OPF_OK
                   : ctx->fail(OPF_EINVAL, "arguments " + std::to_string(a) + " and " +
                                               std::to_string(b) + " must name the same dat");
    };
    rc = same(0, 1);
    if (!rc) rc = same(yslot, yslot + 1);
    if (!rc && adj) rc = same(3, 4);
    if (!rc && flux2) rc = same(2, 3);
    if (!rc && flux2) rc = same(4, 5);
    if (rc) return rc;
    if (want_gbl) {
        rc = check_gbl(ctx, gbls[0], 1, OPF_READ, 0, 0);
        if (rc) return rc;
    }
    // an increment target must not be one of the loop's inputs, by handle or
    // by memory; the adjoint's direct output nbar neither
    for (int k = 0; k < yslot; ++k)
        if (args[k].dat == args[yslot].dat)
            return ctx->fail(OPF_EINVAL, "argument " + std::to_string(yslot) +
                                             " aliases input argument " + std::to_string(k));
    for (int k = 0; k < nargs; ++k) {
        const bool out = args[k].access != OPF_READ;
        if (!out || (k == yslot + 1)) continue;
        for (int j = 0; j < nargs; ++j) {
            // the other map column of the same output is the same dat by design
            if (j == k || (args[j].dat == args[k].dat && args[j].access != OPF_READ)) continue;
            rc = check_disjoint(ctx, args[k].dat, {args[j].dat},
                                ("argument " + std::to_string(k)).c_str());
            if (rc) return rc;
        }
    }
    auto it = ctx->plans.find(m);
    if (it == ctx->plans.end()) return ctx->fail(OPF_ESTATE, "no plan for this map: call opf_plan");
    PlanRec &pr = *it->second;
    if (pr.map_version != mr.version) return ctx->fail(OPF_ESTATE, "plan is stale: map re-declared");
    rc = device_ready(ctx);
    if (rc) return rc;
    if (!pr.on_device) return ctx->fail(OPF_ESTATE, "plan is not on the device");

    const int op = kernel == OPF_K_EDGE_FLUX       ? opf::gpu::OP_FLUX
                   : kernel == OPF_K_EDGE_FLUX_ADJ ? opf::gpu::OP_ADJOINT
                   : kernel == OPF_K_EDGE_SPECRAD  ? opf::gpu::OP_SPECRAD
                   : grad                          ? opf::gpu::OP_GRAD
                                                   : opf::gpu::OP_FLUX2;
    const bool fp32 = T == OPF_F32;
    if (variant == OPF_V_OWNER && !pr.dev.owner_ok)
        return ctx->fail(OPF_EINVAL, "the plan has no owner clusters (cluster_size 0)");
    if (variant == OPF_V_FLAT && pr.dev.nflat <= 0)
        return ctx->fail(OPF_EINVAL, "the map needs more than 128 flat colours");
    if ((variant == OPF_V_COLOURED || variant == OPF_V_COLOURED_LDS_ATOMIC) && !pr.host.coloured_ok)
        return ctx->fail(OPF_EINVAL, "the plan has no two-level colouring (" + pr.host.coloured_why +
                                         "): use the OWNER or ATOMIC variant");
    if (variant != OPF_V_ATOMIC && variant != OPF_V_FLAT) {
        const size_t lds = opf::gpu::edge_lds_bytes(op, fp32, variant, pr.dev.umax, pr.dev.K);
        if (lds > ctx->max_lds)
            return ctx->fail(OPF_EINVAL, "a workgroup needs " + std::to_string(lds) +
                                             " B of LDS; use a smaller block or cluster size");
        if (lds > ctx->lds_limit) {
            int e = opf::gpu::set_lds_limit(ctx->max_lds);
            if (e) return hip_fail(ctx, (hipError_t)e, "raising the LDS limit");
            ctx->lds_limit = ctx->max_lds;
        }
    }
    opf::gpu::EdgeArrays ea;
    const DatRec &q = ctx->dats[args[0].dat];
    for (int c = 0; c < 6; ++c) ea.xin[c] = comp(q, c);
    const DatRec &y = ctx->dats[args[yslot].dat];
    for (int c = 0; c < y.dim; ++c) ea.yout[c] = (double *)comp(y, c);
    if (adj) {
        const DatRec &n = ctx->dats[args[2].dat], &rb = ctx->dats[args[3].dat];
        const DatRec &nb = ctx->dats[args[7].dat];
        for (int c = 0; c < 3; ++c) ea.w[c] = comp(n, c);
        for (int c = 0; c < 6; ++c) ea.xin[6 + c] = comp(rb, c);
        for (int c = 0; c < 3; ++c) ea.wout[c] = (double *)comp(nb, c);
    } else if (flux2) {
        const DatRec &g = ctx->dats[args[2].dat], &vol = ctx->dats[args[4].dat];
        const DatRec &n = ctx->dats[args[6].dat], &dx = ctx->dats[args[7].dat];
        for (int c = 0; c < 18; ++c) ea.xin[6 + c] = comp(g, c);
        ea.xin[24] = comp(vol, 0);
        for (int c = 0; c < 3; ++c) ea.w[c] = comp(n, c);
        for (int c = 0; c < 3; ++c) ea.w[3 + c] = comp(dx, c);
    } else {
        const DatRec &n = ctx->dats[args[2].dat];
        for (int c = 0; c < 3; ++c) ea.w[c] = comp(n, c);
    }
    const double gamma = want_gbl ? *static_cast<const double *>(gbls[0].ptr) : 0.0;
    opf::gpu::LaunchOpts lo;
    lo.overwrite = overwrite ? 1 : 0;
    int e = opf::gpu::launch_edge(op, fp32, variant, pr.dev, ea, gamma, st, lo);
    if (e) return hip_fail(ctx, (hipError_t)e, "edge loop launch");
    return OPF_OK;
}

// Internal label of every user element of set s (identity if not renumbered).
const std::vector<int32_t> *set_perm(const opf_ctx *ctx, opf_set s)
{
    const SetRec &sr = ctx->sets[s];
    if (sr.plan_map < 0) return nullptr;
    auto it = ctx->plans.find(sr.plan_map);
    if (it == ctx->plans.end()) return nullptr;
    const MapRec &m = ctx->maps[sr.plan_map];
    return s == m.to ? &it->second->host.node_new : &it->second->host.edge_new;
}

// The map's entries in the internal numbering of both sets, on the device
// (uploaded once per map version).
int device_map(opf_ctx *ctx, opf_map m, const int32_t *&out)
{
    const MapRec &mr = ctx->maps[m];
    DevMap &dm = ctx->dmaps[m];
    if (dm.ptr && dm.version == mr.version) {
        out = dm.ptr;
        return OPF_OK;
    }
    const int64_t nfrom = ctx->sets[mr.from].size;
    const std::vector<int32_t> *pf = set_perm(ctx, mr.from), *pt = set_perm(ctx, mr.to);
    std::vector<int32_t> v((size_t)nfrom * mr.dim);
    for (int64_t r = 0; r < nfrom; ++r) {
        const int64_t row = pf ? (*pf)[r] : r;
        for (int k = 0; k < mr.dim; ++k) {
            const int32_t x = mr.idx[(size_t)r * mr.dim + k];
            v[(size_t)row * mr.dim + k] = pt ? (*pt)[x] : x;
        }
    }
    ctx->dfree(dm.ptr);
    dm.ptr = static_cast<int32_t *>(ctx->dalloc(v.size() * sizeof(int32_t)));
    if (!dm.ptr) return ctx->fail(OPF_ENOMEM, "device allocation of a map failed");
    hipError_t e = hipMemcpy(dm.ptr, v.data(), v.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(ctx, e, "map upload");
    dm.version = mr.version;
    out = dm.ptr;
    return OPF_OK;
}

void free_tinv(opf_ctx *ctx, DevTetInverse &d)
{
    for (int32_t *p : {d.t2n, d.t2e, d.e2t_off, d.e2t, d.n2t_off, d.n2t, d.n2t_pos, d.ring_off, d.chunk_e,
                       d.halo_off, d.halo, d.vsec_off, d.vsec, d.vloc_off})
        ctx->dfree(p);
    ctx->dfree(d.ring);
    ctx->dfree(d.vloc);
    ctx->dfree(d.scratch);
    ctx->dfree(d.wT);
    ctx->dfree(d.edge_det);
    d = DevTetInverse();
}

// Local edge k of a tet: vertices (p, q) and the completing pair (r, s) such
// that (p, q, r, s) is an even permutation of (0, 1, 2, 3).
const int kLocal[6][4] = {{0, 1, 2, 3}, {0, 2, 3, 1}, {0, 3, 1, 2},
                          {1, 2, 0, 3}, {1, 3, 2, 0}, {2, 3, 0, 1}};

// Host arrays of the ring form (layout in opf::gpu::TetArrays).
struct Rings {
    int KG = 0, nchunk = 0, L = 0, RB = 0, DV = 0;
    std::vector<int32_t> ring_off, chunk_e, halo_off, halo, vsec_off, vsec, vloc_off;
    std::vector<uint16_t> ring, vloc;
};

// Builds the ring form from the plan's internal edge->node map (e2n), the tets
// in internal numbering (tn, 4 per tet) and the CSR list of the tets around
// every edge (eo, el: tet * 8 + local edge, ascending tet order).  Chunks are
// the plan's owner clusters (512 nodes without them).  Returns false, and the
// record form serves, when a chunk's edges are not one contiguous range of
// the edge order, a chunk's nodes and halo exceed kGeoMaxRows, a batch of
// kGeoThreads edges has more than kGeoMaxBatch entries, the edges at a chunk's
// nodes exceed kGeoMaxSlots, or the tets around an edge are not one fan (each
// next tet sharing a face with the last).
bool build_rings(const std::vector<int32_t> &e2n, int64_t N, int64_t E, int KG,
                 const std::vector<int32_t> &tn, const std::vector<int32_t> &eo,
                 const std::vector<int32_t> &el, Rings &R)
{
    if (KG <= 0 || N <= 0 || (int64_t)eo.size() != E + 1) return false;
    if (E + (int64_t)el.size() >= ((int64_t)1 << 31)) return false;
    const int64_t nch = (N + KG - 1) / KG;
    R.KG = KG;
    R.nchunk = (int)nch;
    R.chunk_e.assign(2 * nch, 0);
    std::vector<int64_t> last(nch, -1);
    for (int64_t e = 0; e < E; ++e) {
        const int64_t c = std::min(e2n[2 * e], e2n[2 * e + 1]) / KG;
        if (last[c] < 0) R.chunk_e[2 * c] = (int32_t)e;
        else if (last[c] != e - 1) return false;  // not one contiguous range
        last[c] = e;
        ++R.chunk_e[2 * c + 1];
    }
    // halo of every chunk: the other vertices of its edges' tets, ascending
    std::vector<std::vector<int32_t>> halo(nch);
    std::vector<int32_t> mark(N, -1), loc(N, -1);
    for (int64_t c = 0; c < nch; ++c) {
        const int64_t v0 = c * KG, v1 = std::min<int64_t>(N, v0 + KG);
        std::vector<int32_t> &h = halo[c];
        auto see = [&](int32_t v) {
            if ((v < v0 || v >= v1) && mark[v] != (int32_t)c) {
                mark[v] = (int32_t)c;
                h.push_back(v);
            }
        };
        for (int64_t e = R.chunk_e[2 * c]; e < R.chunk_e[2 * c] + R.chunk_e[2 * c + 1]; ++e) {
            see(e2n[2 * e]);
            see(e2n[2 * e + 1]);
            for (int32_t j = eo[e]; j < eo[e + 1]; ++j) {
                const int32_t t = el[j] >> 3;
                for (int v = 0; v < 4; ++v) see(tn[4 * (int64_t)t + v]);
            }
        }
        std::sort(h.begin(), h.end());
        if (KG + (int64_t)h.size() > opf::gpu::kGeoMaxRows) return false;
        R.L = std::max<int>(R.L, KG + (int)h.size());
    }
    R.halo_off.assign(nch + 1, 0);
    for (int64_t c = 0; c < nch; ++c) R.halo_off[c + 1] = R.halo_off[c] + (int32_t)halo[c].size();
    R.halo.resize(R.halo_off[nch]);
    for (int64_t c = 0; c < nch; ++c)
        std::copy(halo[c].begin(), halo[c].end(), R.halo.begin() + R.halo_off[c]);
    // per edge: a and b, then the chain of the tets around it: vertices
    // c_0 .. c_k such that tet i is (a, b, c_(i-1), c_i), an even permutation of
    // its vertices; a closed ring repeats c_0 at the end (k tets, k + 1 entries)
    R.ring_off.assign(E + 1, 0);
    for (int64_t e = 0; e < E; ++e) R.ring_off[e + 1] = R.ring_off[e] + 3 + (eo[e + 1] - eo[e]);
    R.ring.assign((size_t)R.ring_off[E] + 2, 0);  // +2: the kernel copies whole 4-byte words
    // the ring kernel stages the entries of kGeoThreads edges at a time in LDS
    for (int64_t c = 0; c < nch; ++c) {
        const int64_t e0 = R.chunk_e[2 * c], e1 = e0 + R.chunk_e[2 * c + 1];
        for (int64_t b = e0; b < e1; b += opf::gpu::kGeoThreads) {
            const int64_t n = R.ring_off[std::min<int64_t>(e1, b + opf::gpu::kGeoThreads)] - R.ring_off[b];
            if (n > opf::gpu::kGeoMaxBatch) return false;
            R.RB = std::max<int>(R.RB, (int)n);
        }
    }
    std::vector<int32_t> pr, ps;
    std::vector<uint8_t> used;
    for (int64_t c = 0; c < nch; ++c) {
        const int64_t v0 = c * KG;
        const std::vector<int32_t> &h = halo[c];
        for (size_t i = 0; i < h.size(); ++i) loc[h[i]] = KG + (int32_t)i;
        auto local = [&](int32_t v) -> uint16_t {
            return (uint16_t)(v >= v0 && v < v0 + KG ? v - v0 : loc[v]);
        };
        for (int64_t e = R.chunk_e[2 * c]; e < R.chunk_e[2 * c] + R.chunk_e[2 * c + 1]; ++e) {
            const int32_t a = e2n[2 * e], b = e2n[2 * e + 1];
            const int k = eo[e + 1] - eo[e];
            pr.assign(k, 0);
            ps.assign(k, 0);
            for (int i = 0; i < k; ++i) {
                const int64_t t = el[eo[e] + i] >> 3;
                const int l = el[eo[e] + i] & 7;
                const int32_t *g = &tn[4 * t];
                // (a, b, r, s) even: as listed when a is the local edge's first
                // vertex, else (q, p, s, r)
                const int32_t gp = g[kLocal[l][0]], gq = g[kLocal[l][1]];
                const bool fwd = gp == a;
                if (!(fwd ? gq == b : gq == a && gp == b)) return false;  // t2e disagrees with e2n
                pr[i] = g[kLocal[l][fwd ? 2 : 3]];
                ps[i] = g[kLocal[l][fwd ? 3 : 2]];
            }
            int64_t o = R.ring_off[e];
            R.ring[o++] = local(a);
            R.ring[o++] = local(b);
            if (k == 0) {
                R.ring[o++] = local(a);  // no tets: an empty chain (c_0 only)
                continue;
            }
            // start: the tet whose r is no tet's s (an open fan), else the first
            int start = 0;
            for (int i = 0; i < k; ++i)
                if (std::find(ps.begin(), ps.end(), pr[i]) == ps.end()) {
                    start = i;
                    break;
                }
            used.assign(k, 0);
            used[start] = 1;
            R.ring[o++] = local(pr[start]);
            R.ring[o++] = local(ps[start]);
            int32_t last = ps[start];
            for (int n = 1; n < k; ++n) {
                int next = -1;
                for (int i = 0; i < k && next < 0; ++i)
                    if (!used[i] && pr[i] == last) next = i;
                if (next < 0) return false;  // not one fan of tets around the edge
                used[next] = 1;
                last = ps[next];
                R.ring[o++] = local(last);
            }
        }
    }
    // incident edges of every node, ascending edge order
    std::vector<int32_t> n2e_off(N + 1, 0), n2e(2 * E);
    for (int64_t e = 0; e < E; ++e) {
        ++n2e_off[e2n[2 * e] + 1];
        ++n2e_off[e2n[2 * e + 1] + 1];
    }
    for (int64_t i = 0; i < N; ++i) n2e_off[i + 1] += n2e_off[i];
    {
        std::vector<int32_t> fill(n2e_off.begin(), n2e_off.end() - 1);
        for (int64_t e = 0; e < E; ++e) {
            n2e[fill[e2n[2 * e]]++] = (int32_t)e;
            n2e[fill[e2n[2 * e + 1]]++] = (int32_t)e;
        }
    }
    // the volume kernel's slots: per chunk its own edge range, then the edges
    // it shares with lower chunks (vsec)
    R.vsec_off.assign(nch + 1, 0);
    R.vloc_off = n2e_off;
    R.vloc.resize(2 * E);
    std::vector<int32_t> sec;
    for (int64_t c = 0; c < nch; ++c) {
        const int64_t v0 = c * KG, v1 = std::min<int64_t>(N, v0 + KG);
        const int64_t first = R.chunk_e[2 * c], count = R.chunk_e[2 * c + 1];
        sec.clear();
        for (int64_t i = v0; i < v1; ++i)
            for (int32_t j = n2e_off[i]; j < n2e_off[i + 1]; ++j)
                if (n2e[j] < first || n2e[j] >= first + count) sec.push_back(n2e[j]);
        std::sort(sec.begin(), sec.end());
        sec.erase(std::unique(sec.begin(), sec.end()), sec.end());
        if (count + (int64_t)sec.size() > opf::gpu::kGeoMaxSlots) return false;
        R.DV = std::max<int>(R.DV, (int)(count + sec.size()));
        for (int64_t i = v0; i < v1; ++i)
            for (int32_t j = n2e_off[i]; j < n2e_off[i + 1]; ++j) {
                const int64_t e = n2e[j];
                R.vloc[j] = (uint16_t)(e >= first && e < first + count
                                           ? e - first
                                           : count + (std::lower_bound(sec.begin(), sec.end(), (int32_t)e) - sec.begin()));
            }
        R.vsec_off[c + 1] = R.vsec_off[c] + (int32_t)sec.size();
        R.vsec.insert(R.vsec.end(), sec.begin(), sec.end());
    }
    return true;
}

// The gather form's copies of the tet maps: tets reordered by their lowest
// internal vertex (so that the tets around a node or an edge sit close
// together), both maps in internal numbering, and the CSR lists of the
// (tet, local index) pairs of every edge and node in that tet order,
// packed as tet * 8 + local edge and tet * 4 + local vertex; plus the scratch
// buffer of the per-tet results (kTetScratch doubles per tet).
int tet_inverse(opf_ctx *ctx, opf_map t2n, opf_map t2e, const opf::Plan &P, DevTetInverse *&out)
{
    DevTetInverse &d = ctx->tinv[std::make_pair((int)t2n, (int)t2e)];
    const MapRec &mn = ctx->maps[t2n], &me = ctx->maps[t2e];
    if (d.e2t && d.vn == mn.version && d.ve == me.version) {
        out = &d;
        return OPF_OK;
    }
    const int64_t T = ctx->sets[mn.from].size, N = ctx->sets[mn.to].size,
                  E = ctx->sets[me.to].size;
    if (T * 8 >= ((int64_t)1 << 31)) return ctx->fail(OPF_ESIZE, "too many tets for the gather form");
    const std::vector<int32_t> *pn = set_perm(ctx, mn.to), *pe = set_perm(ctx, me.to);
    // counting sort of the tets by their lowest internal vertex
    std::vector<int64_t> cnt(N + 1, 0);
    std::vector<int32_t> lowest(T);
    for (int64_t t = 0; t < T; ++t) {
        int32_t lo = INT32_MAX;
        for (int v = 0; v < 4; ++v) {
            const int32_t x = mn.idx[t * 4 + v];
            lo = std::min(lo, pn ? (*pn)[x] : x);
        }
        lowest[t] = lo;
        ++cnt[lo + 1];
    }
    for (int64_t i = 0; i < N; ++i) cnt[i + 1] += cnt[i];
    std::vector<int32_t> ord(T);
    for (int64_t t = 0; t < T; ++t) ord[cnt[lowest[t]]++] = (int32_t)t;
    std::vector<int32_t>().swap(lowest);
    std::vector<int32_t> tn(T * 4), te(T * 6);
    for (int64_t k = 0; k < T; ++k) {
        const int64_t t = ord[k];
        for (int v = 0; v < 4; ++v) {
            const int32_t x = mn.idx[t * 4 + v];
            tn[k * 4 + v] = pn ? (*pn)[x] : x;
        }
        for (int j = 0; j < 6; ++j) {
            const int32_t x = me.idx[t * 6 + j];
            te[k * 6 + j] = pe ? (*pe)[x] : x;
        }
    }
    std::vector<int32_t>().swap(ord);
    auto invert = [](const std::vector<int32_t> &m, int dim, int stride, int64_t n,
                     std::vector<int32_t> &off, std::vector<int32_t> &lst) {
        off.assign(n + 1, 0);
        for (int32_t x : m) ++off[x + 1];
        for (int64_t i = 0; i < n; ++i) off[i + 1] += off[i];
        lst.resize(m.size());
        std::vector<int32_t> fill(off.begin(), off.end() - 1);
        for (size_t k = 0; k < m.size(); ++k)  // ascending tet order within each list
            lst[fill[m[k]]++] = (int32_t)((k / dim) * stride + k % dim);
    };
    std::vector<int32_t> eo, el, no, nl;
    invert(te, 6, 8, E, eo, el);
    invert(tn, 4, 4, N, no, nl);
    // the slot of every (tet, vertex) pair in its node's list: the per-tet
    // records of the reverse are written there, so that each node sums a
    // contiguous run
    std::vector<int32_t> npos(4 * T);
    for (size_t j = 0; j < nl.size(); ++j) npos[nl[j]] = (int32_t)j;
    // bit 31 of each local edge: the edge runs from the local edge's second
    // vertex to its first (the map orients it the other way round)
    if ((int64_t)P.e2n.size() != 2 * E) return ctx->fail(OPF_ESTATE, "the edge plan has no map");
    for (int64_t t = 0; t < T; ++t)
        for (int k = 0; k < 6; ++k) {
            const int32_t e = te[6 * t + k];
            if (P.e2n[2 * (int64_t)e] != tn[4 * t + kLocal[k][0]]) te[6 * t + k] = (int32_t)((uint32_t)e | 0x80000000u);
        }
    const int KG = P.owner_ok ? P.cluster_size : 512;
    Rings R;
    const bool rings = build_rings(P.e2n, N, E, KG, tn, eo, el, R);

    free_tinv(ctx, d);
    auto up = [&](const auto &v, auto *&dst) {
        using V = std::remove_const_t<std::remove_reference_t<decltype(v[0])>>;
        dst = static_cast<V *>(ctx->dalloc(v.size() * sizeof(V)));
        if (!dst) return ctx->fail(OPF_ENOMEM, "device allocation of tet incidence failed");
        hipError_t e = hipMemcpy(dst, v.data(), v.size() * sizeof(V), hipMemcpyHostToDevice);
        return e == hipSuccess ? OPF_OK : hip_fail(ctx, e, "tet incidence upload");
    };
    int rc = up(tn, d.t2n);
    if (!rc) rc = up(te, d.t2e);
    if (!rc) rc = up(eo, d.e2t_off);
    if (!rc) rc = up(el, d.e2t);
    if (!rc) rc = up(no, d.n2t_off);
    if (!rc) rc = up(nl, d.n2t);
    if (!rc) rc = up(npos, d.n2t_pos);
    if (!rc && rings) {
        rc = up(R.ring_off, d.ring_off);
        if (!rc) rc = up(R.ring, d.ring);
        if (!rc) rc = up(R.chunk_e, d.chunk_e);
        if (!rc) rc = up(R.halo_off, d.halo_off);
        if (!rc) rc = up(R.halo.empty() ? std::vector<int32_t>(1, 0) : R.halo, d.halo);
        if (!rc) rc = up(R.vsec_off, d.vsec_off);
        if (!rc) rc = up(R.vsec.empty() ? std::vector<int32_t>(1, 0) : R.vsec, d.vsec);
        if (!rc) rc = up(R.vloc_off, d.vloc_off);
        if (!rc) rc = up(R.vloc.empty() ? std::vector<uint16_t>(1, 0) : R.vloc, d.vloc);
        if (!rc) {
            d.edge_det = static_cast<double *>(ctx->dalloc((size_t)std::max<int64_t>(E, 1) * sizeof(double)));
            if (!d.edge_det) rc = ctx->fail(OPF_ENOMEM, "device allocation of the edge sums failed");
        }
        d.nchunk = R.nchunk;
        d.KG = R.KG;
        d.L = R.L;
        d.RB = R.RB;
        d.DV = R.DV;
    }
    if (rc) {
        free_tinv(ctx, d);
        return rc;
    }
    // per-tet records: the reverse's 12 values, and the forward's 19 when the
    // ring form does not serve it
    const size_t per_tet = rings ? 12 : opf::gpu::kTetScratch;
    d.scratch = static_cast<double *>(ctx->dalloc((size_t)T * per_tet * sizeof(double)));
    d.wT = static_cast<double *>(ctx->dalloc((size_t)std::max<int64_t>(E, 1) * 3 * sizeof(double)));
    if (!d.scratch || !d.wT) {
        free_tinv(ctx, d);
        return ctx->fail(OPF_ENOMEM, "device allocation of the tet scratch failed");
    }
    d.vn = mn.version;
    d.ve = me.version;
    out = &d;
    return OPF_OK;
}

int tet_loop(opf_ctx *ctx, int kernel, opf_set s, int nargs, const opf_arg *args, int ngbl,
             const opf_gbl *gbls, int variant, hipStream_t st)
{
    const bool adj = kernel == OPF_K_GEOMETRY_ADJ;
    const int want_args = adj ? 4 : 3;
    if (nargs != want_args || !args)
        return ctx->fail(OPF_EINVAL, "expected " + std::to_string(want_args) + " arguments");
    if (ngbl != 1 || !gbls) return ctx->fail(OPF_EINVAL, "expected one global (period)");
    if (variant != OPF_V_ATOMIC && variant != OPF_V_OWNER)
        return ctx->fail(OPF_EINVAL, "the tet loops run as ATOMIC (scatter) or OWNER (gather)");
    const bool gather = variant == OPF_V_OWNER;
    const opf_map t2n = args[0].map, t2e = args[1].map;
    if (!ctx->map_ok(t2n) || !ctx->map_ok(t2e)) return ctx->fail(OPF_EINVAL, "invalid map");
    const MapRec &mn = ctx->maps[t2n], &me = ctx->maps[t2e];
    if (mn.from != s || mn.dim != 4) return ctx->fail(OPF_EINVAL, "t2n must map the loop set, arity 4");
    if (me.from != s || me.dim != 6) return ctx->fail(OPF_EINVAL, "t2e must map the loop set, arity 6");
    const opf_set nodes = mn.to, edges = me.to;
    const int eplan = ctx->sets[edges].plan_map;
    if (eplan < 0 || ctx->maps[eplan].from != edges || ctx->maps[eplan].to != nodes)
        return ctx->fail(OPF_ESTATE, "the edge set needs a plan of its edge->node map");
    // the forward gather completes every weight and volume in one thread:
    // it may WRITE them instead of incrementing
    auto out_access = [&](int k) {
        if (adj) return (int)OPF_READ;
        return gather && args[k].access == OPF_WRITE ? (int)OPF_WRITE : (int)OPF_INC;
    };
    std::vector<Want> w = {{nodes, OPF_ALL, t2n, 3, OPF_F64, OPF_READ},
                           {edges, OPF_ALL, t2e, 3, OPF_F64, out_access(1)},
                           {nodes, OPF_ALL, t2n, 1, OPF_F64, out_access(2)}};
    if (adj) w.push_back({nodes, OPF_ALL, t2n, 3, OPF_F64, OPF_INC});
    int rc = OPF_OK;
    for (int k = 0; k < nargs && !rc; ++k) rc = check_arg(ctx, args[k], w[k], k);
    if (!rc) rc = check_gbl(ctx, gbls[0], 1, OPF_READ, 0, 0);
    if (rc) return rc;
    const int out0 = adj ? 3 : 1;
    for (int k = out0; k < nargs; ++k)
        for (int j = 0; j < out0; ++j)
            if (args[k].dat == args[j].dat)
                return ctx->fail(OPF_EINVAL, "an incremented argument aliases an input");
    // by memory as well: every incremented dat against every other argument
    for (int k = out0; k < nargs && !rc; ++k)
        for (int j = 0; j < nargs && !rc; ++j)
            if (j != k) rc = check_disjoint(ctx, args[k].dat, {args[j].dat}, "tet loop");
    if (rc) return rc;
    const double period = *static_cast<const double *>(gbls[0].ptr);
    if (!(period >= 0.0)) return ctx->fail(OPF_EINVAL, "period must be >= 0");
    auto it = ctx->plans.find(eplan);
    if (it == ctx->plans.end()) return ctx->fail(OPF_ESTATE, "no plan for the edge map");
    if (it->second->map_version != ctx->maps[eplan].version)
        return ctx->fail(OPF_ESTATE, "the edge map's plan is stale");
    rc = device_ready(ctx);
    if (rc) return rc;
    if (!it->second->on_device) return ctx->fail(OPF_ESTATE, "plan is not on the device");
    opf::gpu::TetArrays ta;
    if (gather) {
        DevTetInverse *inv = nullptr;
        rc = tet_inverse(ctx, t2n, t2e, it->second->host, inv);
        if (!rc) {
            ta.t2n = inv->t2n;
            ta.t2e = inv->t2e;
            ta.e2t_off = inv->e2t_off;
            ta.e2t = inv->e2t;
            ta.n2t_off = inv->n2t_off;
            ta.n2t = inv->n2t;
            ta.n2t_pos = inv->n2t_pos;
            ta.scratch = inv->scratch;
            ta.wT = inv->wT;
            ta.ring_off = inv->ring_off;
            ta.ring = inv->ring;
            ta.chunk_e = reinterpret_cast<const int2 *>(inv->chunk_e);
            ta.halo_off = inv->halo_off;
            ta.halo = inv->halo;
            ta.vsec_off = inv->vsec_off;
            ta.vsec = inv->vsec;
            ta.vloc_off = inv->vloc_off;
            ta.vloc = inv->vloc;
            ta.DV = inv->DV;
            ta.edge_det = inv->edge_det;
            ta.nchunk = inv->nchunk;
            ta.KG = inv->KG;
            ta.L = inv->L;
            ta.RB = inv->RB;
        }
    } else {
        rc = device_map(ctx, t2n, ta.t2n);
        if (!rc) rc = device_map(ctx, t2e, ta.t2e);
    }
    if (rc) return rc;
    ta.N = (int)ctx->sets[nodes].size;
    ta.E = (int)ctx->sets[edges].size;
    ta.e2n = it->second->dev.e2n;
    const DatRec &x = ctx->dats[args[0].dat], &wd = ctx->dats[args[1].dat];
    const DatRec &vd = ctx->dats[args[2].dat];
    for (int d = 0; d < 3; ++d) {
        ta.x[d] = static_cast<const double *>(comp(x, d));
        ta.w[d] = (double *)comp(wd, d);
    }
    ta.vol = (double *)comp(vd, 0);
    if (!adj) {
        ta.write_w = args[1].access == OPF_WRITE ? 1 : 0;
        ta.write_vol = args[2].access == OPF_WRITE ? 1 : 0;
    }
    if (adj) {
        const DatRec &xb = ctx->dats[args[3].dat];
        for (int d = 0; d < 3; ++d) ta.xbar[d] = (double *)comp(xb, d);
    }
    const int64_t T = ctx->sets[s].size;
    if (gather) {
        rc = scratch_begin(ctx, st);
        if (rc) return rc;
    }
    int e = opf::gpu::launch_geometry(adj, gather, (int)T, ta, period, st);
    if (e) return hip_fail(ctx, (hipError_t)e, "tet loop launch");
    return gather ? scratch_end(ctx, st) : OPF_OK;
}

int direct_loop(opf_ctx *ctx, int kernel, opf_set s, int nargs, const opf_arg *args, int ngbl,
                const opf_gbl *gbls, hipStream_t st)
{
    int rc = OPF_OK;
    if (kernel == OPF_K_RK_STAGE) {
        if ((nargs != 4 && nargs != 5) || !args)
            return ctx->fail(OPF_EINVAL, "expected 4 arguments (5 with local time steps)");
        if (ngbl != 2 || !gbls) return ctx->fail(OPF_EINVAL, "expected 2 globals");
        if (!ctx->dat_ok(args[0].dat)) return ctx->fail(OPF_EINVAL, "argument 0: invalid dat");
        const int T = ctx->dats[args[0].dat].type;
        const bool keep_res = args[1].access == OPF_READ;
        const Want w[5] = {{s, -1, OPF_ID, 6, T, OPF_READ},
                           {s, -1, OPF_ID, 6, OPF_F64, keep_res ? OPF_READ : OPF_RW},
                           {s, -1, OPF_ID, 1, OPF_F64, OPF_READ},
                           {s, -1, OPF_ID, 6, T, OPF_WRITE},
                           {s, -1, OPF_ID, 1, OPF_F64, OPF_READ}};
        for (int k = 0; k < nargs && !rc; ++k) rc = check_arg(ctx, args[k], w[k], k);
        if (!rc) rc = check_gbl(ctx, gbls[0], 1, OPF_READ, 0, 0);
        if (!rc) rc = check_gbl(ctx, gbls[1], 6, OPF_INC, 1, 1);
        if (rc) return rc;
        if (args[0].dat == args[3].dat || args[1].dat == args[3].dat)
            return ctx->fail(OPF_EINVAL, "q must not alias q0 or res");
        const opf_dat dtd = nargs == 5 ? args[4].dat : -1;
        rc = check_disjoint(ctx, args[3].dat, {args[0].dat, args[1].dat, args[2].dat, dtd}, "RK stage q");
        if (!rc && !keep_res)
            rc = check_disjoint(ctx, args[1].dat, {args[0].dat, args[2].dat, dtd}, "RK stage res");
        if (!rc)
            rc = check_gbl_disjoint(ctx, gbls[1].ptr, 6 * sizeof(double),
                                    {args[0].dat, args[1].dat, args[2].dat, args[3].dat, dtd},
                                    "RK stage ss");
        if (rc) return rc;
        rc = device_ready(ctx);
        if (rc) return rc;
        rc = scratch_begin(ctx, st);
        if (rc) return rc;
        opf::gpu::NodeArrays na;
        const DatRec &q0 = ctx->dats[args[0].dat], &res = ctx->dats[args[1].dat];
        const DatRec &vol = ctx->dats[args[2].dat], &q = ctx->dats[args[3].dat];
        for (int c = 0; c < 6; ++c) {
            na.q0[c] = comp(q0, c);
            na.res[c] = (double *)comp(res, c);
            na.q[c] = (void *)comp(q, c);
        }
        na.vol = static_cast<const double *>(vol.ptr);
        if (nargs == 5) na.dt = static_cast<const double *>(ctx->dats[args[4].dat].ptr);
        const double adt = *static_cast<const double *>(gbls[0].ptr);
        int e = opf::gpu::launch_rk_stage(T == OPF_F32, (int)ctx->sets[s].size, na, adt,
                                          static_cast<double *>(gbls[1].ptr), ctx->scratch,
                                          keep_res, st);
        if (e) return hip_fail(ctx, (hipError_t)e, "RK stage launch");
        return scratch_end(ctx, st);
    }
    if (kernel == OPF_K_LOCAL_DT) {
        if (nargs != 3 || !args) return ctx->fail(OPF_EINVAL, "expected 3 arguments");
        if (ngbl != 1 || !gbls) return ctx->fail(OPF_EINVAL, "expected 1 global");
        const Want w[3] = {{s, -1, OPF_ID, 1, OPF_F64, OPF_READ},
                           {s, -1, OPF_ID, 1, OPF_F64, OPF_READ},
                           {s, -1, OPF_ID, 1, OPF_F64, OPF_WRITE}};
        for (int k = 0; k < 3 && !rc; ++k) rc = check_arg(ctx, args[k], w[k], k);
        if (!rc) rc = check_gbl(ctx, gbls[0], 1, OPF_READ, 0, 0);
        if (rc) return rc;
        if (args[2].dat == args[0].dat || args[2].dat == args[1].dat)
            return ctx->fail(OPF_EINVAL, "dt must not alias vol or lam");
        rc = check_disjoint(ctx, args[2].dat, {args[0].dat, args[1].dat}, "local time step dt");
        if (rc) return rc;
        rc = device_ready(ctx);
        if (rc) return rc;
        const double cfl = *static_cast<const double *>(gbls[0].ptr);
        int e = opf::gpu::launch_local_dt((int)ctx->sets[s].size,
                                          static_cast<const double *>(ctx->dats[args[0].dat].ptr),
                                          static_cast<const double *>(ctx->dats[args[1].dat].ptr),
                                          cfl, static_cast<double *>(ctx->dats[args[2].dat].ptr), st);
        if (e) return hip_fail(ctx, (hipError_t)e, "local time-step launch");
        return OPF_OK;
    }
    // DT_MIN
    if (nargs != 2 || !args) return ctx->fail(OPF_EINVAL, "expected 2 arguments");
    if (ngbl != 2 || !gbls) return ctx->fail(OPF_EINVAL, "expected 2 globals");
    const Want w[2] = {{s, -1, OPF_ID, 1, OPF_F64, OPF_READ}, {s, -1, OPF_ID, 1, OPF_F64, OPF_READ}};
    for (int k = 0; k < 2 && !rc; ++k) rc = check_arg(ctx, args[k], w[k], k);
    if (!rc) rc = check_gbl(ctx, gbls[0], 1, OPF_READ, 0, 0);
    if (!rc) rc = check_gbl(ctx, gbls[1], 1, OPF_MIN, 1, 1);
    if (!rc)
        rc = check_gbl_disjoint(ctx, gbls[1].ptr, sizeof(double), {args[0].dat, args[1].dat}, "time step");
    if (rc) return rc;
    rc = device_ready(ctx);
    if (rc) return rc;
    rc = scratch_begin(ctx, st);
    if (rc) return rc;
    const double cfl = *static_cast<const double *>(gbls[0].ptr);
    int e = opf::gpu::launch_dt_min((int)ctx->sets[s].size,
                                    static_cast<const double *>(ctx->dats[args[0].dat].ptr),
                                    static_cast<const double *>(ctx->dats[args[1].dat].ptr), cfl,
                                    static_cast<double *>(gbls[1].ptr), ctx->scratch, st);
    if (e) return hip_fail(ctx, (hipError_t)e, "time-step launch");
    return scratch_end(ctx, st);
}

}  // namespace

extern "C" {

int opf_init(opf_ctx **out, int hip_device)
{
    if (!out) return OPF_EINVAL;
    *out = nullptr;
    std::unique_ptr<opf_ctx> ctx(new (std::nothrow) opf_ctx());
    if (!ctx) return OPF_ENOMEM;
    if (hip_device < -1) return OPF_EINVAL;
    if (hip_device >= 0) {
        int n = 0;
        if (hipGetDeviceCount(&n) != hipSuccess || hip_device >= n) return OPF_EDEVICE;
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) return OPF_EDEVICE;
        ctx->max_lds = prop.sharedMemPerBlock;
        ctx->lds_limit = prop.sharedMemPerBlock;
        if (prop.sharedMemPerBlockOptin > ctx->max_lds) ctx->max_lds = prop.sharedMemPerBlockOptin;
        if (resolve_static_scratch(hip_device) != OPF_OK) return OPF_EDEVICE;
    }
    ctx->err.reserve(512);  // error messages of later calls need no allocation
    ctx->device = hip_device;
    *out = ctx.release();
    return OPF_OK;
}

int opf_finalize(opf_ctx *ctx)
{
    if (!ctx) return OPF_OK;
    if (ctx->device >= 0) {
        (void)hipSetDevice(ctx->device);
        (void)hipDeviceSynchronize();
        for (auto &kv : ctx->plans) free_plan(ctx, *kv.second);
        for (auto &kv : ctx->dmaps) ctx->dfree(kv.second.ptr);
        for (auto &kv : ctx->tinv) free_tinv(ctx, kv.second);
        ctx->dfree(ctx->scratch);
        if (ctx->scratch_ev) (void)hipEventDestroy(ctx->scratch_ev);
    }
    delete ctx;
    return OPF_OK;
}

const char *opf_last_error(const opf_ctx *ctx) { return ctx ? ctx->err.c_str() : "no context"; }

int opf_set_allocator(opf_ctx *ctx, void *(*alloc_fn)(void *, size_t), void (*free_fn)(void *, void *),
                      void *user)
{
    if (!ctx) return OPF_EINVAL;
    if (!ctx->plans.empty() || ctx->scratch)
        return ctx->fail(OPF_ESTATE, "set the allocator before the first plan or loop");
    if ((alloc_fn == nullptr) != (free_fn == nullptr))
        return ctx->fail(OPF_EINVAL, "give both allocator functions or neither");
    ctx->alloc_fn = alloc_fn;
    ctx->free_fn = free_fn;
    ctx->alloc_user = user;
    return OPF_OK;
}

int opf_decl_set(opf_ctx *ctx, int64_t size, const char *name, opf_set *out)
{
    if (!ctx || !out) return ctx ? ctx->fail(OPF_EINVAL, "out is NULL") : OPF_EINVAL;
    if (size <= 0 || size >= ((int64_t)1 << 29))
        return ctx->fail(OPF_ESIZE, "set size must be in (0, 2^29)");
    SetRec s;
    s.size = size;
    s.name = name ? name : "";
    ctx->sets.push_back(s);
    *out = (opf_set)ctx->sets.size() - 1;
    return OPF_OK;
}

int opf_decl_map(opf_ctx *ctx, opf_set from, opf_set to, int dim, const int32_t *idx, int index_base,
                 const char *name, opf_map *out)
{
    if (!ctx) return OPF_EINVAL;
    if (!out || !idx) return ctx->fail(OPF_EINVAL, "NULL argument");
    if (!ctx->set_ok(from) || !ctx->set_ok(to)) return ctx->fail(OPF_EINVAL, "invalid set handle");
    if (dim < 1) return ctx->fail(OPF_EINVAL, "map dimension must be >= 1");
    if (index_base != 0 && index_base != 1) return ctx->fail(OPF_EINVAL, "index_base must be 0 or 1");
    // a map declared again under its name must join the same sets with the
    // same arity: handles other code holds keep their meaning
    if (name && *name)
        for (const MapRec &m : ctx->maps)
            if (m.name == name && (m.from != from || m.to != to || m.dim != dim))
                return ctx->fail(OPF_EINVAL, std::string("map '") + name +
                                                 "' already joins other sets or has another arity");
    if (ctx->sets[from].plan_map >= 0 || ctx->sets[to].plan_map >= 0) {
        // a map declared on renumbered sets would have to be in internal
        // numbering; keep declarations in user numbering only
        std::string nm = name ? name : "";
        bool replacing = false;
        for (const MapRec &m : ctx->maps)
            if (!nm.empty() && m.name == nm) replacing = true;
        if (!replacing) return ctx->fail(OPF_ESTATE, "declare maps before planning their sets");
    }
    const int64_t n = ctx->sets[from].size * dim, tsz = ctx->sets[to].size;
    std::vector<int32_t> v(idx, idx + n);
    for (int64_t k = 0; k < n; ++k) {
        v[k] -= index_base;
        if (v[k] < 0 || v[k] >= tsz)
            return ctx->fail(OPF_ERANGE, "map entry " + std::to_string(k) + " = " +
                                             std::to_string(idx[k]) + " is outside the target set");
    }
    MapRec m;
    m.from = from;
    m.to = to;
    m.dim = dim;
    m.idx.swap(v);
    m.name = name ? name : "";
    m.version = ctx->next_version++;
    if (!m.name.empty())
        for (size_t k = 0; k < ctx->maps.size(); ++k)
            if (ctx->maps[k].name == m.name) {
                ctx->maps[k] = std::move(m);  // the old plan becomes stale
                *out = (opf_map)k;
                return OPF_OK;
            }
    ctx->maps.push_back(std::move(m));
    *out = (opf_map)ctx->maps.size() - 1;
    return OPF_OK;
}

int opf_plan(opf_ctx *ctx, opf_map map, const opf_plan_opts *opts, opf_plan_info *info)
{
    if (!ctx) return OPF_EINVAL;
    if (!ctx->map_ok(map)) return ctx->fail(OPF_EINVAL, "invalid map handle");
    MapRec &m = ctx->maps[map];
    if (m.dim != 2) return ctx->fail(OPF_EINVAL, "plans are built for arity-2 (edge) maps");
    for (opf_set s : {m.from, m.to})
        if (ctx->sets[s].plan_map >= 0 && ctx->sets[s].plan_map != map)
            return ctx->fail(OPF_ESTATE, "set '" + ctx->sets[s].name + "' is renumbered by another plan");
    opf::PlanOptions po;
    if (opts) {
        po.renumber = opts->renumber;
        po.block_size = opts->block_size;
        po.colour_sort = opts->colour_sort;
        po.cluster_size = opts->cluster_size;
        po.lane_groups = opts->lane_groups;
        po.bank_spread = opts->bank_spread;
        po.halo_order = opts->halo_order;
        po.coords = opts->coords;
    }
    auto t0 = std::chrono::steady_clock::now();
    auto pr = std::unique_ptr<PlanRec>(new (std::nothrow) PlanRec());
    if (!pr) return ctx->fail(OPF_ENOMEM, "out of host memory");
    int rc;
    try {
        rc = opf::build_plan(ctx->sets[m.to].size, ctx->sets[m.from].size, m.idx.data(), po,
                             pr->host, ctx->err);
    } catch (const std::bad_alloc &) {
        return ctx->fail(OPF_ENOMEM, "out of host memory while planning");
    }
    if (rc) return rc;
    opf::VerifyResult vr = opf::verify_plan(pr->host, m.idx.data());
    if (!vr.ok)
        return ctx->fail(OPF_EPLAN, "plan property " + std::to_string(vr.property) + ": " + vr.message);
    pr->map_version = m.version;
    auto old = ctx->plans.find(map);
    if (old != ctx->plans.end() || !ctx->dmaps.empty() || !ctx->tinv.empty()) {
        if (ctx->device >= 0) {
            (void)hipSetDevice(ctx->device);
            (void)hipDeviceSynchronize();
        }
        // the device copies of the tet maps are in the internal numbering this
        // plan is about to change: drop them (rebuilt on their next use)
        for (auto &kv : ctx->dmaps) ctx->dfree(kv.second.ptr);
        ctx->dmaps.clear();
        for (auto &kv : ctx->tinv) free_tinv(ctx, kv.second);
        ctx->tinv.clear();
    }
    if (old != ctx->plans.end()) {
        free_plan(ctx, *old->second);
        ctx->plans.erase(old);
    }
    if (ctx->device >= 0) {
        rc = upload_plan(ctx, *pr);
        if (rc) return rc;
    }
    double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    ctx->sets[m.from].plan_map = map;
    ctx->sets[m.to].plan_map = map;
    if (info) {
        const opf::Plan &P = pr->host;
        info->nblocks = P.nblocks();
        info->nblock_colours = P.nblock_colours;
        info->max_elem_colours = P.max_elem_colours;
        info->mean_elem_colours = P.mean_elem_colours;
        info->sum_unique = (int64_t)P.uniq.size();
        info->max_unique = P.max_unique;
        info->min_blocks_per_colour = P.min_blocks_per_colour;
        info->bandwidth_before = P.bandwidth_before;
        info->bandwidth_after = P.bandwidth_after;
        info->plan_seconds = secs;
        info->device_bytes = pr->device_bytes;
        info->nclusters = P.nclusters();
        info->owner_edge_visits = P.owner_edge_visits;
        info->max_cluster_segments = P.max_cluster_segments;
        info->owner_ok = P.owner_ok ? 1 : 0;
        info->owner_compact = P.owner_ok ? 1 : 0;
        info->flat_colours = P.flat_colours;
        info->flat_ok = P.flat_ok ? 1 : 0;
        info->coloured_ok = P.coloured_ok ? 1 : 0;
    }
    ctx->plans[map] = std::move(pr);
    return OPF_OK;
}

int opf_get_perm(const opf_ctx *ctx, opf_set s, int32_t *new_of_old)
{
    if (!ctx || !new_of_old || !ctx->set_ok(s)) return OPF_EINVAL;
    const SetRec &sr = ctx->sets[s];
    if (sr.plan_map < 0) {
        for (int64_t i = 0; i < sr.size; ++i) new_of_old[i] = (int32_t)i;
        return OPF_OK;
    }
    auto it = ctx->plans.find(sr.plan_map);
    if (it == ctx->plans.end()) return OPF_ESTATE;
    const MapRec &m = ctx->maps[sr.plan_map];
    const std::vector<int32_t> &p = (s == m.to) ? it->second->host.node_new : it->second->host.edge_new;
    std::memcpy(new_of_old, p.data(), p.size() * sizeof(int32_t));
    return OPF_OK;
}

int opf_plan_view_get(const opf_ctx *ctx, opf_map map, opf_plan_view *out)
{
    if (!ctx || !out || !ctx->map_ok(map)) return OPF_EINVAL;
    auto it = ctx->plans.find(map);
    if (it == ctx->plans.end()) return OPF_ESTATE;
    const opf::Plan &P = it->second->host;
    out->nnodes = P.N;
    out->nedges = P.E;
    out->nblocks = P.nblocks();
    out->nblock_colours = P.nblock_colours;
    out->block_size = P.block_size;
    out->e2n = P.e2n.data();
    out->block_offsets = P.block_off.data();
    out->block_colour = P.block_colour.data();
    out->colour_blocks = P.colour_blocks.data();
    out->colour_offsets = P.colour_off.data();
    out->elem_colour = P.ecol.data();
    out->block_ncolours = P.block_ncol.data();
    out->unique_offsets = P.uniq_off.data();
    out->unique_nodes = P.uniq.data();
    out->local_idx = P.lidx.data();
    out->cluster_size = P.cluster_size;
    out->nclusters = P.nclusters();
    out->cluster_seg_offsets = P.cl_seg_off.data();
    out->cluster_seg_start = P.cl_seg_start.data();
    out->cluster_seg_len = P.cl_seg_len.data();
    out->cluster_range = P.cl_prim.data();
    out->cluster_list_offsets = P.cl_sec_off.data();
    out->cluster_list_edges = P.cl_sec_eid.data();
    out->nflat_colours = P.flat_ok ? P.flat_colours : 0;
    out->flat_offsets = P.flat_ok ? P.flat_off.data() : nullptr;
    out->flat_edges = P.flat_ok ? P.flat_eid.data() : nullptr;
    out->owner_swap = P.owner_swap.empty() ? nullptr : P.owner_swap.data();
    if (!P.coloured_ok) {  // no two-level colouring: its arrays are absent
        out->block_colour = nullptr;
        out->colour_blocks = nullptr;
        out->colour_offsets = nullptr;
        out->elem_colour = nullptr;
        out->block_ncolours = nullptr;
        out->unique_offsets = nullptr;
        out->unique_nodes = nullptr;
        out->local_idx = nullptr;
    }
    out->cluster_interior = P.cl_nint.data();
    out->cluster_cut_offsets = P.cl_cut_off.data();
    out->cluster_cut_edges = P.cl_cut_eid.data();
    out->cluster_cut_ends = P.cl_cut_end.data();
    out->cluster_cutf_edges = P.cl_cutf_eid.data();
    out->cluster_cutf_ends = P.cl_cutf_end.data();
    return OPF_OK;
}

int opf_plan_verify(const opf_ctx *ctx, opf_map map, opf_plan_report *report)
{
    if (!ctx || !ctx->map_ok(map)) return OPF_EINVAL;
    auto it = ctx->plans.find(map);
    if (it == ctx->plans.end()) return OPF_ESTATE;
    opf::VerifyResult vr = opf::verify_plan(it->second->host, ctx->maps[map].idx.data());
    if (report) {
        report->ok = vr.ok ? 1 : 0;
        report->property = vr.property;
        report->where = vr.where;
        std::snprintf(report->message, sizeof report->message, "%s", vr.message.c_str());
    }
    return vr.ok ? OPF_OK : OPF_EPLAN;
}

int opf_decl_dat(opf_ctx *ctx, opf_set s, int dim, int type, void *dev_ptr, int64_t ld,
                 const char *name, opf_dat *out)
{
    if (!ctx) return OPF_EINVAL;
    if (!out || !ctx->set_ok(s)) return ctx->fail(OPF_EINVAL, "invalid set handle or out");
    if (dim < 1) return ctx->fail(OPF_EINVAL, "dat dimension must be >= 1");
    if (type != OPF_F64 && type != OPF_F32) return ctx->fail(OPF_ETYPE, "unknown dat type");
    if (!dev_ptr && ctx->device >= 0) return ctx->fail(OPF_EINVAL, "NULL device pointer");
    if (ld < ctx->sets[s].size) return ctx->fail(OPF_ESIZE, "leading dimension below the set size");
    DatRec d;
    d.set = s;
    d.dim = dim;
    d.type = type;
    d.ptr = dev_ptr;
    d.ld = ld;
    d.name = name ? name : "";
    ctx->dats.push_back(d);
    *out = (opf_dat)ctx->dats.size() - 1;
    return OPF_OK;
}

int opf_par_loop(opf_ctx *ctx, int kernel, opf_set s, int nargs, const opf_arg *args, int ngbl,
                 const opf_gbl *gbls, int variant, void *stream)
{
    if (!ctx) return OPF_EINVAL;
    if (!ctx->set_ok(s)) return ctx->fail(OPF_EINVAL, "invalid set handle");
    ctx->err.clear();
    hipStream_t st = static_cast<hipStream_t>(stream);
    switch (kernel) {
    case OPF_K_EDGE_FLUX:
    case OPF_K_EDGE_FLUX_ADJ:
    case OPF_K_EDGE_SPECRAD:
    case OPF_K_EDGE_GRAD:
    case OPF_K_EDGE_FLUX2: return edge_loop(ctx, kernel, s, nargs, args, ngbl, gbls, variant, st);
    case OPF_K_RK_STAGE:
    case OPF_K_DT_MIN:
    case OPF_K_LOCAL_DT: return direct_loop(ctx, kernel, s, nargs, args, ngbl, gbls, st);
    case OPF_K_GEOMETRY:
    case OPF_K_GEOMETRY_ADJ: return tet_loop(ctx, kernel, s, nargs, args, ngbl, gbls, variant, st);
    default: return ctx->fail(OPF_EINVAL, "unknown kernel");
    }
}

int opf_edge_flux(opf_ctx *ctx, opf_set edges, opf_map e2n, opf_dat q, opf_dat n, opf_dat res,
                  double gamma, int variant, int res_access, void *stream)
{
    if (!ctx) return OPF_EINVAL;
    if (!ctx->dat_ok(q) || !ctx->dat_ok(n) || !ctx->dat_ok(res))
        return ctx->fail(OPF_EINVAL, "invalid dat handle");
    const int T = ctx->dats[q].type, TN = ctx->dats[n].type;
    const opf_arg a[5] = {{q, 0, e2n, 6, T, OPF_READ},
                          {q, 1, e2n, 6, T, OPF_READ},
                          {n, -1, OPF_ID, 3, TN, OPF_READ},
                          {res, 0, e2n, 6, OPF_F64, res_access},
                          {res, 1, e2n, 6, OPF_F64, res_access}};
    const opf_gbl g[1] = {{&gamma, 1, OPF_F64, OPF_READ, 0}};
    return opf_par_loop(ctx, OPF_K_EDGE_FLUX, edges, 5, a, 1, g, variant, stream);
}

int opf_edge_flux_adjoint(opf_ctx *ctx, opf_set edges, opf_map e2n, opf_dat q, opf_dat n,
                          opf_dat rbar, opf_dat qbar, opf_dat nbar, double gamma, int variant,
                          int qbar_access, void *stream)
{
    if (!ctx) return OPF_EINVAL;
    if (!ctx->dat_ok(q) || !ctx->dat_ok(n)) return ctx->fail(OPF_EINVAL, "invalid dat handle");
    const int T = ctx->dats[q].type, TN = ctx->dats[n].type;
    const opf_arg a[8] = {{q, 0, e2n, 6, T, OPF_READ},          {q, 1, e2n, 6, T, OPF_READ},
                          {n, -1, OPF_ID, 3, TN, OPF_READ},       {rbar, 0, e2n, 6, OPF_F64, OPF_READ},
                          {rbar, 1, e2n, 6, OPF_F64, OPF_READ},   {qbar, 0, e2n, 6, OPF_F64, qbar_access},
                          {qbar, 1, e2n, 6, OPF_F64, qbar_access}, {nbar, -1, OPF_ID, 3, OPF_F64, OPF_WRITE}};
    const opf_gbl g[1] = {{&gamma, 1, OPF_F64, OPF_READ, 0}};
    return opf_par_loop(ctx, OPF_K_EDGE_FLUX_ADJ, edges, 8, a, 1, g, variant, stream);
}

int opf_edge_specrad(opf_ctx *ctx, opf_set edges, opf_map e2n, opf_dat q, opf_dat n, opf_dat lam,
                     double gamma, int variant, void *stream)
{
    if (!ctx) return OPF_EINVAL;
    if (!ctx->dat_ok(q) || !ctx->dat_ok(n)) return ctx->fail(OPF_EINVAL, "invalid dat handle");
    const int T = ctx->dats[q].type, TN = ctx->dats[n].type;
    const opf_arg a[5] = {{q, 0, e2n, 6, T, OPF_READ},
                          {q, 1, e2n, 6, T, OPF_READ},
                          {n, -1, OPF_ID, 3, TN, OPF_READ},
                          {lam, 0, e2n, 1, OPF_F64, OPF_INC},
                          {lam, 1, e2n, 1, OPF_F64, OPF_INC}};
    const opf_gbl g[1] = {{&gamma, 1, OPF_F64, OPF_READ, 0}};
    return opf_par_loop(ctx, OPF_K_EDGE_SPECRAD, edges, 5, a, 1, g, variant, stream);
}

int opf_rk_stage(opf_ctx *ctx, opf_set nodes, opf_dat q0, opf_dat res, opf_dat vol, opf_dat q,
                 double alpha_dt, double *ss_dev, int res_access, void *stream)
{
    if (!ctx) return OPF_EINVAL;
    if (!ctx->dat_ok(q0)) return ctx->fail(OPF_EINVAL, "invalid dat handle");
    const int T = ctx->dats[q0].type;
    const opf_arg a[4] = {{q0, -1, OPF_ID, 6, T, OPF_READ},
                          {res, -1, OPF_ID, 6, OPF_F64, res_access},
                          {vol, -1, OPF_ID, 1, OPF_F64, OPF_READ},
                          {q, -1, OPF_ID, 6, T, OPF_WRITE}};
    const opf_gbl g[2] = {{&alpha_dt, 1, OPF_F64, OPF_READ, 0}, {ss_dev, 6, OPF_F64, OPF_INC, 1}};
    return opf_par_loop(ctx, OPF_K_RK_STAGE, nodes, 4, a, 2, g, OPF_V_COLOURED, stream);
}

int opf_edge_gradient(opf_ctx *ctx, opf_set edges, opf_map e2n, opf_dat q, opf_dat n, opf_dat G,
                      int variant, int g_access, void *stream)
{
    if (!ctx) return OPF_EINVAL;
    const opf_arg a[5] = {{q, 0, e2n, 6, OPF_F64, OPF_READ},
                          {q, 1, e2n, 6, OPF_F64, OPF_READ},
                          {n, -1, OPF_ID, 3, OPF_F64, OPF_READ},
                          {G, 0, e2n, 18, OPF_F64, g_access},
                          {G, 1, e2n, 18, OPF_F64, g_access}};
    return opf_par_loop(ctx, OPF_K_EDGE_GRAD, edges, 5, a, 0, nullptr, variant, stream);
}

int opf_edge_flux2(opf_ctx *ctx, opf_set edges, opf_map e2n, opf_dat q, opf_dat G, opf_dat vol,
                   opf_dat n, opf_dat dx, opf_dat res, double gamma, int variant, int res_access,
                   void *stream)
{
    if (!ctx) return OPF_EINVAL;
    const opf_arg a[10] = {{q, 0, e2n, 6, OPF_F64, OPF_READ},
                           {q, 1, e2n, 6, OPF_F64, OPF_READ},
                           {G, 0, e2n, 18, OPF_F64, OPF_READ},
                           {G, 1, e2n, 18, OPF_F64, OPF_READ},
                           {vol, 0, e2n, 1, OPF_F64, OPF_READ},
                           {vol, 1, e2n, 1, OPF_F64, OPF_READ},
                           {n, -1, OPF_ID, 3, OPF_F64, OPF_READ},
                           {dx, -1, OPF_ID, 3, OPF_F64, OPF_READ},
                           {res, 0, e2n, 6, OPF_F64, res_access},
                           {res, 1, e2n, 6, OPF_F64, res_access}};
    const opf_gbl g[1] = {{&gamma, 1, OPF_F64, OPF_READ, 0}};
    return opf_par_loop(ctx, OPF_K_EDGE_FLUX2, edges, 10, a, 1, g, variant, stream);
}

}  // extern "C"

namespace {

// The fused edge loop + stage.  noalloc: the per-cluster partials go to the
// static device scratch of the current device instead of the plan's buffer, and
// nothing is allocated (no context scratch, no event): the allocation-free entry
// point.
int edge_flux_stage(opf_ctx *ctx, opf_set edges, opf_map e2n, opf_dat q, opf_dat n, opf_dat q0,
                    opf_dat vol, opf_dat dt, opf_dat qout, double gamma, double alpha,
                    double *ss_dev, void *stream, bool noalloc)
{
    if (!ctx) return OPF_EINVAL;
    ctx->err.clear();
    if (!ctx->set_ok(edges) || !ctx->map_ok(e2n)) return ctx->fail(OPF_EINVAL, "invalid handle");
    const MapRec &mr = ctx->maps[e2n];
    if (mr.dim != 2 || mr.from != edges)
        return ctx->fail(OPF_EINVAL, "the loop set must be the source set of an arity-2 map");
    const opf_set nodes = mr.to;
    if (!ctx->dat_ok(q)) return ctx->fail(OPF_EINVAL, "argument 0: invalid dat");
    const int T = ctx->dats[q].type;
    if (T != OPF_F64 && T != OPF_F32) return ctx->fail(OPF_ETYPE, "argument 0: unknown type");
    const opf_arg a[7] = {{q, 0, e2n, 6, T, OPF_READ},         {n, -1, OPF_ID, 3, T, OPF_READ},
                          {q0, -1, OPF_ID, 6, T, OPF_READ},    {vol, -1, OPF_ID, 1, OPF_F64, OPF_READ},
                          {qout, -1, OPF_ID, 6, T, OPF_WRITE}, {dt, -1, OPF_ID, 1, OPF_F64, OPF_READ},
                          {q, 1, e2n, 6, T, OPF_READ}};
    const Want w[7] = {{nodes, 0, e2n, 6, T, OPF_READ},         {edges, -1, OPF_ID, 3, T, OPF_READ},
                       {nodes, -1, OPF_ID, 6, T, OPF_READ},     {nodes, -1, OPF_ID, 1, OPF_F64, OPF_READ},
                       {nodes, -1, OPF_ID, 6, T, OPF_WRITE},    {nodes, -1, OPF_ID, 1, OPF_F64, OPF_READ},
                       {nodes, 1, e2n, 6, T, OPF_READ}};
    int rc = OPF_OK;
    for (int k = 0; k < 7 && !rc; ++k) {
        if (k == 5 && dt < 0) continue;  // no per-node step
        rc = check_arg(ctx, a[k], w[k], k);
    }
    if (rc) return rc;
    if (qout == q || qout == q0) return ctx->fail(OPF_EINVAL, "qout must not alias q or q0");
    if (!ss_dev) return ctx->fail(OPF_EINVAL, "ss must be device memory");
    rc = check_disjoint(ctx, qout, {q, n, q0, vol, dt}, "fused stage qout");
    if (!rc)
        rc = check_gbl_disjoint(ctx, ss_dev, 6 * sizeof(double), {q, n, q0, vol, dt, qout},
                                "fused stage ss");
    if (rc) return rc;
    auto it = ctx->plans.find(e2n);
    if (it == ctx->plans.end()) return ctx->fail(OPF_ESTATE, "no plan for this map: call opf_plan");
    PlanRec &pr = *it->second;
    if (pr.map_version != mr.version) return ctx->fail(OPF_ESTATE, "plan is stale: map re-declared");
    if (!pr.host.owner_ok) return ctx->fail(OPF_EINVAL, "the fused loop needs owner clusters");
    double *partial = pr.dev.stage_partial;
    if (noalloc) {
        rc = device_bind(ctx);
        if (rc) return rc;
        if (pr.on_device && pr.dev.ncl > opf::gpu::kStaticMaxClusters)
            return ctx->fail(OPF_ESIZE, "the allocation-free fused loop holds at most 16384 "
                                        "clusters; this plan has more");
        partial = static_scratch_of(ctx->device);
        if (!partial) return ctx->fail(OPF_ESTATE, "static scratch not resolved for this device");
    } else {
        rc = device_ready(ctx);
        if (rc) return rc;
    }
    if (!pr.on_device) return ctx->fail(OPF_ESTATE, "plan is not on the device");
    const bool fp32 = T == OPF_F32;
    const size_t lds = opf::gpu::edge_lds_bytes(opf::gpu::OP_FLUX, fp32, OPF_V_OWNER, pr.dev.umax,
                                                pr.dev.K);
    if (lds > ctx->max_lds)
        return ctx->fail(OPF_EINVAL, "a workgroup needs " + std::to_string(lds) + " B of LDS");
    if (lds > ctx->lds_limit) {
        int e = opf::gpu::set_lds_limit(ctx->max_lds);
        if (e) return hip_fail(ctx, (hipError_t)e, "raising the LDS limit");
        ctx->lds_limit = ctx->max_lds;
    }
    opf::gpu::EdgeArrays ea;
    const DatRec &qd = ctx->dats[q], &nd = ctx->dats[n];
    for (int c = 0; c < 6; ++c) ea.xin[c] = comp(qd, c);
    for (int c = 0; c < 3; ++c) ea.w[c] = comp(nd, c);
    opf::gpu::NodeArrays na;
    const DatRec &q0d = ctx->dats[q0], &qod = ctx->dats[qout];
    for (int c = 0; c < 6; ++c) {
        na.q0[c] = comp(q0d, c);
        na.q[c] = (void *)comp(qod, c);
    }
    na.vol = static_cast<const double *>(ctx->dats[vol].ptr);
    if (dt >= 0) na.dt = static_cast<const double *>(ctx->dats[dt].ptr);
    opf::gpu::LaunchOpts lo;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    if (noalloc) {
        const int e = opf::gpu::launch_edge_stage(fp32, pr.dev, ea, na, gamma, alpha, ss_dev,
                                                  partial, st, lo);
        return e ? hip_fail(ctx, (hipError_t)e, "fused loop launch") : OPF_OK;
    }
    rc = scratch_begin(ctx, st);
    if (rc) return rc;
    int e = opf::gpu::launch_edge_stage(fp32, pr.dev, ea, na, gamma, alpha, ss_dev, partial, st, lo);
    if (e) return hip_fail(ctx, (hipError_t)e, "fused loop launch");
    return scratch_end(ctx, st);
}

}  // namespace

extern "C" {

int opf_edge_flux_stage(opf_ctx *ctx, opf_set edges, opf_map e2n, opf_dat q, opf_dat n,
                        opf_dat q0, opf_dat vol, opf_dat dt, opf_dat qout, double gamma,
                        double alpha, double *ss_dev, void *stream)
{
    return edge_flux_stage(ctx, edges, e2n, q, n, q0, vol, dt, qout, gamma, alpha, ss_dev, stream,
                           false);
}

int opf_edge_flux_stage_noalloc(opf_ctx *ctx, opf_set edges, opf_map e2n, opf_dat q, opf_dat n,
                                opf_dat q0, opf_dat vol, opf_dat dt, opf_dat qout, double gamma,
                                double alpha, double *ss_dev, void *stream)
{
    return edge_flux_stage(ctx, edges, e2n, q, n, q0, vol, dt, qout, gamma, alpha, ss_dev, stream,
                           true);
}

int opf_geometry(opf_ctx *ctx, opf_set tets, opf_map t2n, opf_map t2e, opf_dat x, double period,
                 opf_dat w, opf_dat vol, int variant, void *stream)
{
    if (!ctx) return OPF_EINVAL;
    const opf_arg a[3] = {{x, OPF_ALL, t2n, 3, OPF_F64, OPF_READ},
                          {w, OPF_ALL, t2e, 3, OPF_F64, OPF_INC},
                          {vol, OPF_ALL, t2n, 1, OPF_F64, OPF_INC}};
    const opf_gbl g[1] = {{&period, 1, OPF_F64, OPF_READ, 0}};
    return opf_par_loop(ctx, OPF_K_GEOMETRY, tets, 3, a, 1, g, variant, stream);
}

int opf_geometry_adjoint(opf_ctx *ctx, opf_set tets, opf_map t2n, opf_map t2e, opf_dat x,
                         double period, opf_dat wbar, opf_dat volbar, opf_dat xbar, int variant,
                         void *stream)
{
    if (!ctx) return OPF_EINVAL;
    const opf_arg a[4] = {{x, OPF_ALL, t2n, 3, OPF_F64, OPF_READ},
                          {wbar, OPF_ALL, t2e, 3, OPF_F64, OPF_READ},
                          {volbar, OPF_ALL, t2n, 1, OPF_F64, OPF_READ},
                          {xbar, OPF_ALL, t2n, 3, OPF_F64, OPF_INC}};
    const opf_gbl g[1] = {{&period, 1, OPF_F64, OPF_READ, 0}};
    return opf_par_loop(ctx, OPF_K_GEOMETRY_ADJ, tets, 4, a, 1, g, variant, stream);
}

int opf_rk_stage_local(opf_ctx *ctx, opf_set nodes, opf_dat q0, opf_dat res, opf_dat vol,
                       opf_dat dt, opf_dat q, double alpha, double *ss_dev, int res_access,
                       void *stream)
{
    if (!ctx) return OPF_EINVAL;
    if (!ctx->dat_ok(q0)) return ctx->fail(OPF_EINVAL, "invalid dat handle");
    const int T = ctx->dats[q0].type;
    const opf_arg a[5] = {{q0, -1, OPF_ID, 6, T, OPF_READ},
                          {res, -1, OPF_ID, 6, OPF_F64, res_access},
                          {vol, -1, OPF_ID, 1, OPF_F64, OPF_READ},
                          {q, -1, OPF_ID, 6, T, OPF_WRITE},
                          {dt, -1, OPF_ID, 1, OPF_F64, OPF_READ}};
    const opf_gbl g[2] = {{&alpha, 1, OPF_F64, OPF_READ, 0}, {ss_dev, 6, OPF_F64, OPF_INC, 1}};
    return opf_par_loop(ctx, OPF_K_RK_STAGE, nodes, 5, a, 2, g, OPF_V_COLOURED, stream);
}

int opf_local_dt(opf_ctx *ctx, opf_set nodes, opf_dat vol, opf_dat lam, double cfl, opf_dat dt,
                 void *stream)
{
    if (!ctx) return OPF_EINVAL;
    const opf_arg a[3] = {{vol, -1, OPF_ID, 1, OPF_F64, OPF_READ},
                          {lam, -1, OPF_ID, 1, OPF_F64, OPF_READ},
                          {dt, -1, OPF_ID, 1, OPF_F64, OPF_WRITE}};
    const opf_gbl g[1] = {{&cfl, 1, OPF_F64, OPF_READ, 0}};
    return opf_par_loop(ctx, OPF_K_LOCAL_DT, nodes, 3, a, 1, g, OPF_V_COLOURED, stream);
}

int opf_dt_min(opf_ctx *ctx, opf_set nodes, opf_dat vol, opf_dat lam, double cfl, double *dt_dev,
               void *stream)
{
    if (!ctx) return OPF_EINVAL;
    const opf_arg a[2] = {{vol, -1, OPF_ID, 1, OPF_F64, OPF_READ}, {lam, -1, OPF_ID, 1, OPF_F64, OPF_READ}};
    const opf_gbl g[2] = {{&cfl, 1, OPF_F64, OPF_READ, 0}, {dt_dev, 1, OPF_F64, OPF_MIN, 1}};
    return opf_par_loop(ctx, OPF_K_DT_MIN, nodes, 2, a, 2, g, OPF_V_COLOURED, stream);
}

int opf_sync(opf_ctx *ctx, void *stream)
{
    if (!ctx) return OPF_EINVAL;
    if (ctx->device < 0) return ctx->fail(OPF_EDEVICE, "host-only context");
    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess) e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e == hipSuccess) e = hipGetLastError();
    return e == hipSuccess ? OPF_OK : hip_fail(ctx, e, "stream synchronise");
}

int opf_check_finite(opf_ctx *ctx, const double *dev_ptr, int n, void *stream)
{
    if (!ctx) return OPF_EINVAL;
    if (!dev_ptr || n < 1 || n > 4096) return ctx->fail(OPF_EINVAL, "bad pointer or count");
    if (ctx->device < 0) return ctx->fail(OPF_EDEVICE, "host-only context");
    std::vector<double> h(n);
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(h.data(), dev_ptr, n * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(ctx, e, "reading the reduction");
    for (int k = 0; k < n; ++k)
        if (!std::isfinite(h[k]))
            return ctx->fail(OPF_ENONFINITE, "value " + std::to_string(k) + " is not finite");
    return OPF_OK;
}

}  // extern "C"
