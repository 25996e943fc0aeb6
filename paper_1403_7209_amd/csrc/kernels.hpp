// kernels.hpp -- launch interface of the gfx950 kernels (internal to libopflux).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace opf {
namespace gpu {

enum EdgeOpKind { OP_FLUX = 0, OP_ADJOINT = 1, OP_SPECRAD = 2, OP_GRAD = 3, OP_FLUX2 = 4 };

constexpr int kMaxNodeIn = 25;   // node inputs of one edge loop (q, G, vol)
constexpr int kMaxNodeOut = 18;  // node increments (Green-Gauss sums)
constexpr int kMaxEdgeIn = 6;    // direct edge inputs (n, dx)

// Execution variants of an edge loop (values match opf_variant).
enum Variant { V_COLOURED = 0, V_ATOMIC = 1, V_OWNER = 2, V_COLOURED_LDS_ATOMIC = 3, V_FLAT = 4 };

constexpr int kOwnerThreads = 512;

// Device copy of an execution plan (internal numbering, int32 offsets).
struct DevPlan {
    int N = 0, E = 0, nb = 0, nc = 0, umax = 0, block_size = 0;
    const int2 *e2n = nullptr;           // [E] endpoint pairs
    const int *block_off = nullptr;      // [nb+1]
    const int *uniq_off = nullptr;       // [nb+1]
    const int *uniq = nullptr;           // [sum U]
    const uint32_t *lidx = nullptr;      // [E] two 16-bit local indices
    const uint8_t *ecol = nullptr;       // [E]
    const int *block_ncol = nullptr;     // [nb]
    const int *colour_blocks = nullptr;  // [nb]
    std::vector<int> colour_off;         // host copy [nc+1]
    // owner clusters (cluster c owns internal nodes [c K, (c+1) K)), two loops
    // per cluster: the interior block, edges iblk[c].x .. iblk[c].x + iblk[c].y
    // with both ends in c, read through iw; then the cut visits
    // cv_off[c] .. cv_off[c+1], one (edge, owned end) pair each
    int K = 0, ncl = 0;
    bool owner_ok = false;
    const int2 *iblk = nullptr;      // [ncl] (first edge, count)
    const uint32_t *iw = nullptr;    // [E] interior edges: offsets of the first (bits
                                     // 0-12) and second (bits 16-28) end in the
                                     // cluster; bit 31: update the second end first
    const int *cv_off = nullptr;     // [ncl+1]
    const int *cv_eid = nullptr;     // edge of each cut visit
    const int *cv_oth = nullptr;     // its other end (internal node), bit 31 set when
                                     // the owned end is the edge's second node
    const uint16_t *cv_own = nullptr; // offset of the owned end in the cluster
    // the same visits ordered by foreign node within each run (same offsets)
    const int *cvf_eid = nullptr, *cvf_oth = nullptr;
    const uint16_t *cvf_own = nullptr;
    // flat colouring: colour c runs edges flat_eid[flat_off[c] .. flat_off[c+1])
    double *stage_partial = nullptr;  // kSumTail + [ncl][6]: partial sums of the fused stage
    int nflat = 0;
    std::vector<int64_t> flat_off;  // host copy [nflat+1]
    const int *flat_eid = nullptr;  // [E]
};

// Component pointers of the arrays an edge loop touches (SoA: one pointer per
// component, each already offset by component * ld).
struct EdgeArrays {
    const void *xin[kMaxNodeIn] = {};  // node inputs (q; then rbar, or G and vol)
    double *yout[kMaxNodeOut] = {};    // node increments (res, qbar, lambda or G)
    const void *w[kMaxEdgeIn] = {};    // edge inputs (weights n; then dx)
    double *wout[3] = {};              // direct edge outputs (nbar)
};

struct LaunchOpts {
    int xcd_remap = 1;  // give each XCD a contiguous range of partitions/clusters
    int overwrite = 0;  // owner variant: res = sum instead of res += sum
};

// Returns 0 or a hipError_t value.
int launch_edge(int op, bool fp32, int variant, const DevPlan &plan, const EdgeArrays &a,
                double gamma, hipStream_t stream, const LaunchOpts &lo);

struct NodeArrays {
    const void *q0[6] = {};
    double *res[6] = {};
    const double *vol = nullptr;
    void *q[6] = {};
    const double *dt = nullptr;  // per-node time steps, or null for one global step
};

// Buffers of partial sums (the stage reductions): kSumTail doubles, then 6
// per row.  The second pass sums the rows in kSumGroups workgroups, each over
// a fixed block of rows in a fixed order, into the first 6 * kSumGroups
// doubles; the last workgroup to finish (a counter in the next word) adds
// those in order.  The counter must be zero before the first use of a buffer
// and is zero again after every pass.
constexpr int kSumGroups = 16;
constexpr int kSumTail = 6 * kSumGroups + 2;

// q = q0 - alpha_dt * res / vol (alpha_dt * dt_i with per-node steps),
// ss[v] += sum res^2 (two passes, deterministic), res = 0 unless keep_res.
// `partial` holds kSumTail + kRkBlocks * 6 doubles.
constexpr int kRkThreads = 256;
constexpr int kRkBlocks = 2048;
int launch_rk_stage(bool fp32, int N, const NodeArrays &a, double alpha_dt, double *ss,
                    double *partial, bool keep_res, hipStream_t stream);

// The owner FP64/FP32 edge-flux loop with the stage update fused into it:
// q = q0 - adt * res / vol (adt * dt_i when a.dt is set) for every node, and
// ss[v] += sum res^2 (per-cluster partials, fixed-order second pass); the
// residual is never written.  The plan must have owner clusters.  `partial`
// holds kSumTail + 6 * P.ncl doubles (counter zero); every cluster writes its
// six before they are summed.
int launch_edge_stage(bool fp32, const DevPlan &P, const EdgeArrays &a, const NodeArrays &na,
                      double gamma, double adt, double *ss, double *partial, hipStream_t stream,
                      const LaunchOpts &lo);

// Clusters whose partial sums fit the library's static device scratch (the
// fused stage for callers that cannot allocate): 6 doubles each, 768 KiB,
// after the kSumTail doubles of the second pass.
constexpr int kStaticMaxClusters = 16384;

// Device address of that static scratch on the current device (each GPU holds
// its own copy).  Returns 0 or a hipError_t value.
int static_scratch_address(double **out);

// dt = min(dt, cfl * min_i vol_i / lam_i); `partial` holds kSumTail +
// kRkBlocks doubles (the rows after the tail).
int launch_dt_min(int N, const double *vol, const double *lam, double cfl, double *dt,
                  double *partial, hipStream_t stream);

// Tet loops.  t2n [4T] and t2e [6T] in internal numbering; e2n orients the
// edges.  Pointers are SoA components.
struct TetArrays {
    const int *t2n = nullptr;
    const int *t2e = nullptr;
    const int2 *e2n = nullptr;
    // gather form: incident tets of every edge (tet * 8 + local edge) and of
    // every node (tet * 4 + local vertex), CSR in internal numbering; n2t_pos:
    // the index in n2t of every (tet, vertex) pair (tet * 4 + vertex).  In the
    // gather form's t2e, bit 31 marks an edge that runs from the local edge's
    // second vertex to its first.
    const int *e2t_off = nullptr, *e2t = nullptr;
    const int *n2t_off = nullptr, *n2t = nullptr, *n2t_pos = nullptr;
    double *scratch = nullptr;  // gather form: kTetScratch x T doubles
    double *wT = nullptr;       // gather reverse: wbar interleaved, 3 x E doubles
    // ring form of the forward gather (ring != nullptr): node chunks of KG
    // consecutive internal nodes; chunk c owns the edges chunk_e[c] = (first,
    // count) whose smaller end it holds.  Edge e's entries are
    // ring[ring_off[e] .. ring_off[e+1]): a and b (a -> b the edge's
    // orientation), then the chain c_0 .. c_k of the k tets around it, tet i
    // being (a, b, c_(i-1), c_i), an even permutation of its vertices (a
    // closed ring ends with c_k = c_0); all in the chunk's local numbering: its
    // own nodes at 0 .. KG-1, then its halo nodes halo[halo_off[c] ..] at KG,
    // KG + 1, ...  L = KG + the largest halo.  The array has two spare entries
    // at its end.
    const int *ring_off = nullptr;
    const uint16_t *ring = nullptr;
    const int2 *chunk_e = nullptr;
    const int *halo_off = nullptr, *halo = nullptr;
    // volumes: per chunk the edges with their larger end in it and smaller end
    // in a lower chunk (vsec[vsec_off[c] ..], ascending); per node i its edges'
    // slots vloc[vloc_off[i] .. vloc_off[i+1]) in ascending edge order, slot j
    // < count being the chunk's edge first + j, slot count + m its m-th vsec
    // edge.  DV: the most slots of a chunk.
    const int *vsec_off = nullptr, *vsec = nullptr, *vloc_off = nullptr;
    const uint16_t *vloc = nullptr;
    double *edge_det = nullptr;  // per edge: sum of 6 vol over its tets
    int nchunk = 0, KG = 0, L = 0;
    int RB = 0;  // ring entries of the largest batch of kGeoThreads edges of a chunk
    int DV = 0;
    int write_w = 0, write_vol = 0;  // gather forward: WRITE instead of INC
    int N = 0, E = 0;
    const double *x[3] = {};
    double *w[3] = {};      // GEOMETRY: weights (INC); ADJ: wbar (read)
    double *vol = nullptr;  // GEOMETRY: volumes (INC); ADJ: volbar (read)
    double *xbar[3] = {};   // ADJ only
};
// Per-tet results of the gather form: 6 signed face vectors (18 values at
// 18 t) + 1 volume determinant (at 18 T + t) forward, or in reverse the 4
// vertex shares of x-bar, each 3 values at 3 n2t_pos[4 t + v] (node-major).
constexpr int kTetScratch = 19;
// gather = false: one thread per tet, FP64 atomics (summation order varies);
// gather = true: one thread per tet writes its results to the scratch
// buffer, then one thread per edge (weights) and per node (volumes, reverse)
// sums them over the incident tets in a fixed order (deterministic, no atomics).
int launch_geometry(bool adjoint, bool gather, int T, const TetArrays &a, double period,
                    hipStream_t stream);
// The largest L (chunk nodes + halo) the ring kernel takes (24 B of LDS per
// node).
constexpr int kGeoMaxRows = 4096;
// The ring kernel's workgroup: one edge per thread per batch.
constexpr int kGeoThreads = 512;
// Ring words (4 bytes) each thread of the ring kernel prefetches for the next
// batch, and so the most ring entries of one batch.
constexpr int kGeoPre = 8;
constexpr int kGeoMaxBatch = 2 * (kGeoPre * kGeoThreads - 2);
// The volume kernel's workgroup and its most slots per chunk (LDS: 8 B each).
constexpr int kGeoVolThreads = 512;
constexpr int kGeoMaxSlots = 8192;
// LDS bytes of one ring-kernel workgroup: coordinates, then the batch's
// entries (whole 4-byte words, one spare at each end).
inline size_t geo_ring_lds(int L, int RB) { return (size_t)L * 24 + ((size_t)RB / 2 + 2) * 4; }

// dt[i] = cfl * vol[i] / lam[i].
int launch_local_dt(int N, const double *vol, const double *lam, double cfl, double *dt,
                    hipStream_t stream);

// LDS bytes (dynamic and static) of one workgroup of an edge loop.
size_t edge_lds_bytes(int op, bool fp32, int variant, int umax, int K);

// Lets every edge kernel instance use up to `bytes` of LDS in total.
int set_lds_limit(size_t bytes);

}  // namespace gpu
}  // namespace opf
