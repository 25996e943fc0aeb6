// geometry.hip -- the median-dual geometry loop over tets and its reverse.
//
// Inside a tet (p, q, r, s) the dual face between the cells of p and q joins
// the edge midpoint, the centroids of the faces pqr and pqs and the tet
// centroid; its area vector is half the cross product of that quadrilateral's
// diagonals, (x_r + x_s - x_p - x_q) x (x_s - x_r) / 24, pointing from p to q
// when (p, q, r, s) has the tet's orientation.  Each vertex owns a quarter of
// the tet's volume.  These are the edge weights and node volumes that the edge
// loops read (the per-edge data of the edge loops, Sec. 4); computing them on
// the device, and their reverse, lets the flux adjoint's weight sensitivities
// reach the node coordinates.
//
// Two forms.  Scatter: one thread per tet adds its six face vectors and four
// volume quarters (or, in reverse, its four x-bar shares) to HBM with FP64
// atomics.  Gather: no atomics, fixed summation orders, the same bits on every
// run.  The forward gather walks the tets around each edge from coordinates
// staged in LDS (ring form, below); the reverse (and the forward, where a
// mesh does not fit the ring form) writes per-tet results to a scratch buffer
// that one thread per edge or node then sums over its incident tets.  The
// loop runs once per mesh (or once per design step for the reverse).
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace opf {
namespace gpu {
namespace {

// Local edge k: vertices (a, b) and the completing pair (r, s) such that
// (a, b, r, s) is an even permutation of (0, 1, 2, 3).
constexpr int kTetEdge[6][4] = {{0, 1, 2, 3}, {0, 2, 3, 1}, {0, 3, 1, 2},
                                   {1, 2, 0, 3}, {1, 3, 2, 0}, {2, 3, 0, 1}};

__device__ __forceinline__ void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

__device__ __forceinline__ void tet_x(const TetArrays &a, const int *g, double period, double x[4][3])
{
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int d = 0; d < 3; ++d) x[v][d] = a.x[d][g[v]];
    if (period > 0.0) {
        const double ip = 1.0 / period;
#pragma unroll
        for (int v = 1; v < 4; ++v)
#pragma unroll
            for (int d = 0; d < 3; ++d) x[v][d] -= period * rint((x[v][d] - x[0][d]) * ip);
    }
}

// +1 if edge e runs from node na to node nb, else -1 (the map guarantees it
// is one of the two).
__device__ __forceinline__ double orient(const int2 *e2n, int e, int na)
{
    return e2n[e].x == na ? 1.0 : -1.0;
}

__global__ __launch_bounds__(256) void k_geometry(int T, TetArrays a, double period)
{
    const int t = (int)blockIdx.x * 256 + (int)threadIdx.x;
    if (t >= T) return;
    int g[4], ed[6];
#pragma unroll
    for (int v = 0; v < 4; ++v) g[v] = a.t2n[4 * t + v];
#pragma unroll
    for (int k = 0; k < 6; ++k) ed[k] = a.t2e[6 * t + k];
    double x[4][3];
    tet_x(a, g, period, x);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int p = kTetEdge[k][0], q = kTetEdge[k][1], r = kTetEdge[k][2], s = kTetEdge[k][3];
        double u[3], v[3], c[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            u[d] = x[r][d] + x[s][d] - x[p][d] - x[q][d];
            v[d] = x[s][d] - x[r][d];
        }
        cross3(u, v, c);
        const double sg = orient(a.e2n, ed[k], g[p]) * (1.0 / 24.0);
#pragma unroll
        for (int d = 0; d < 3; ++d) unsafeAtomicAdd(a.w[d] + ed[k], sg * c[d]);
    }
    double e1[3], e2[3], e3[3], c[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        e1[d] = x[1][d] - x[0][d];
        e2[d] = x[2][d] - x[0][d];
        e3[d] = x[3][d] - x[0][d];
    }
    cross3(e2, e3, c);
    const double q4 = (e1[0] * c[0] + e1[1] * c[1] + e1[2] * c[2]) * (1.0 / 24.0);
#pragma unroll
    for (int v = 0; v < 4; ++v) unsafeAtomicAdd(a.vol + g[v], q4);
}

__global__ __launch_bounds__(256) void k_geometry_adj(int T, TetArrays a, double period)
{
    const int t = (int)blockIdx.x * 256 + (int)threadIdx.x;
    if (t >= T) return;
    int g[4], ed[6];
#pragma unroll
    for (int v = 0; v < 4; ++v) g[v] = a.t2n[4 * t + v];
#pragma unroll
    for (int k = 0; k < 6; ++k) ed[k] = a.t2e[6 * t + k];
    double x[4][3], xb[4][3];
    tet_x(a, g, period, x);
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int d = 0; d < 3; ++d) xb[v][d] = 0.0;
    // face vector c = u x v / 24: ubar = v x cbar / 24, vbar = cbar x u / 24
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int p = kTetEdge[k][0], q = kTetEdge[k][1], r = kTetEdge[k][2], s = kTetEdge[k][3];
        const double sg = orient(a.e2n, ed[k], g[p]) * (1.0 / 24.0);
        double u[3], v[3], cb[3], ub[3], vb[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            u[d] = x[r][d] + x[s][d] - x[p][d] - x[q][d];
            v[d] = x[s][d] - x[r][d];
            cb[d] = sg * a.w[d][ed[k]];
        }
        cross3(v, cb, ub);
        cross3(cb, u, vb);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            xb[p][d] -= ub[d];
            xb[q][d] -= ub[d];
            xb[r][d] += ub[d] - vb[d];
            xb[s][d] += ub[d] + vb[d];
        }
    }
    // volume V = e1 . (e2 x e3) / 6 with e_k = x_k - x_0, a quarter to each vertex
    const double Vb = 0.25 * (a.vol[g[0]] + a.vol[g[1]] + a.vol[g[2]] + a.vol[g[3]]) * (1.0 / 6.0);
    double e1[3], e2[3], e3[3], c1[3], c2[3], c3[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        e1[d] = x[1][d] - x[0][d];
        e2[d] = x[2][d] - x[0][d];
        e3[d] = x[3][d] - x[0][d];
    }
    cross3(e2, e3, c1);
    cross3(e3, e1, c2);
    cross3(e1, e2, c3);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        xb[1][d] += Vb * c1[d];
        xb[2][d] += Vb * c2[d];
        xb[3][d] += Vb * c3[d];
        xb[0][d] -= Vb * (c1[d] + c2[d] + c3[d]);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int d = 0; d < 3; ++d) unsafeAtomicAdd(a.xbar[d] + g[v], xb[v][d]);
}

// ---------------------------------------------------------- gather form -- */
//
// Phase 1, one thread per tet (tets in the order of the incidence lists, so
// the map reads coalesce): the tet's results go to the scratch buffer as one
// record per tet.  Phase 2, one thread per edge or node: the sum over its
// incident tets, in list order; the tets around an edge or a node are close
// in that order, so their records share cache lines.

// record of tet t: the signed face vector of local edge k / 24 at
// scratch[18 t + 3k + d]; the volume determinant / 24 at scratch[18 T + t] (an
// array of its own, so that the per-node sums read 16 tets per cache line)
__global__ __launch_bounds__(256) void k_tet_forward(int T, TetArrays a, double period)
{
    const int t = (int)blockIdx.x * 256 + (int)threadIdx.x;
    if (t >= T) return;
    int g[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) g[v] = a.t2n[4 * t + v];
    double x[4][3];
    tet_x(a, g, period, x);
    double *rec = a.scratch + (size_t)t * 18;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int p = kTetEdge[k][0], q = kTetEdge[k][1], r = kTetEdge[k][2], s = kTetEdge[k][3];
        double u[3], v[3], c[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            u[d] = x[r][d] + x[s][d] - x[p][d] - x[q][d];
            v[d] = x[s][d] - x[r][d];
        }
        cross3(u, v, c);
        const double sg = (a.t2e[6 * t + k] < 0 ? -1.0 : 1.0) * (1.0 / 24.0);
#pragma unroll
        for (int d = 0; d < 3; ++d) rec[3 * k + d] = sg * c[d];
    }
    double e1[3], e2[3], e3[3], c[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        e1[d] = x[1][d] - x[0][d];
        e2[d] = x[2][d] - x[0][d];
        e3[d] = x[3][d] - x[0][d];
    }
    cross3(e2, e3, c);
    a.scratch[(size_t)18 * T + t] = (e1[0] * c[0] + e1[1] * c[1] + e1[2] * c[2]) * (1.0 / 24.0);
}

// The sums below walk a list in order; they fetch kSumAhead entries at a
// time (these loops are latency-bound) and add them in list order.
constexpr int kSumAhead = 4;

// w[e] += sum over the tets around e of their face vector of e
__global__ __launch_bounds__(256) void k_edge_sum_faces(TetArrays a)
{
    const int e = (int)blockIdx.x * 256 + (int)threadIdx.x;
    if (e >= a.E) return;
    double acc[3] = {0.0, 0.0, 0.0};
    const int end = a.e2t_off[e + 1];
    for (int j = a.e2t_off[e]; j < end; j += kSumAhead) {
        double r[kSumAhead][3];
#pragma unroll
        for (int u = 0; u < kSumAhead; ++u) {
            // past the end of the list: re-read its first entry (always valid)
            const int tk = a.e2t[j + u < end ? j + u : j];
            const double *rec = a.scratch + (size_t)(tk >> 3) * 18 + 3 * (tk & 7);
#pragma unroll
            for (int d = 0; d < 3; ++d) r[u][d] = rec[d];
        }
#pragma unroll
        for (int u = 0; u < kSumAhead; ++u)
#pragma unroll
            for (int d = 0; d < 3; ++d)
                if (j + u < end) acc[d] += r[u][d];
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) a.w[d][e] = (a.write_w ? 0.0 : a.w[d][e]) + acc[d];
}

// vol[i] += sum over the tets around i of a quarter of their volume
__global__ __launch_bounds__(256) void k_node_sum_vol(int T, TetArrays a)
{
    const int i = (int)blockIdx.x * 256 + (int)threadIdx.x;
    if (i >= a.N) return;
    const double *det = a.scratch + (size_t)18 * T;
    double acc = 0.0;
    const int end = a.n2t_off[i + 1];
    for (int j = a.n2t_off[i]; j < end; j += kSumAhead) {
        double r[kSumAhead];
#pragma unroll
        for (int u = 0; u < kSumAhead; ++u) {
            r[u] = det[a.n2t[j + u < end ? j + u : j] >> 2];
        }
#pragma unroll
        for (int u = 0; u < kSumAhead; ++u)
            if (j + u < end) acc += r[u];
    }
    a.vol[i] = (a.write_vol ? 0.0 : a.vol[i]) + acc;
}

// The reverse of one tet at coordinates x (unwrapped): its x-bar shares xb
// from the signed weight adjoints cb[k] = +-wbar / 24 of its six local edges
// and the sum vbs of its vertices' volume adjoints (a quarter of the volume
// to each vertex).  Face c = u x v / 24: ubar = v x cbar, vbar = cbar x u.
__device__ __forceinline__ void tet_shares(const double (&x)[4][3], const double (&cb)[6][3],
                                           double vbs, double (&xb)[4][3])
{
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int d = 0; d < 3; ++d) xb[v][d] = 0.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int p = kTetEdge[k][0], q = kTetEdge[k][1], r = kTetEdge[k][2], s = kTetEdge[k][3];
        double u[3], v[3], ub[3], vb[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            u[d] = x[r][d] + x[s][d] - x[p][d] - x[q][d];
            v[d] = x[s][d] - x[r][d];
        }
        cross3(v, cb[k], ub);
        cross3(cb[k], u, vb);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            xb[p][d] -= ub[d];
            xb[q][d] -= ub[d];
            xb[r][d] += ub[d] - vb[d];
            xb[s][d] += ub[d] + vb[d];
        }
    }
    // volume V = e1 . (e2 x e3) / 6 with e_k = x_k - x_0
    const double Vb = 0.25 * vbs * (1.0 / 6.0);
    double e1[3], e2[3], e3[3], c1[3], c2[3], c3[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        e1[d] = x[1][d] - x[0][d];
        e2[d] = x[2][d] - x[0][d];
        e3[d] = x[3][d] - x[0][d];
    }
    cross3(e2, e3, c1);
    cross3(e3, e1, c2);
    cross3(e1, e2, c3);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        xb[1][d] += Vb * c1[d];
        xb[2][d] += Vb * c2[d];
        xb[3][d] += Vb * c3[d];
        xb[0][d] -= Vb * (c1[d] + c2[d] + c3[d]);
    }
}

// the six weight adjoints of tet t, read from their interleaved copy wT
__device__ __forceinline__ void tet_wbar(const TetArrays &a, int t, double (&cb)[6][3])
{
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int ew = a.t2e[6 * t + k], ed = ew & 0x7fffffff;
        const double sg = (ew < 0 ? -1.0 : 1.0) * (1.0 / 24.0);
#pragma unroll
        for (int d = 0; d < 3; ++d) cb[k][d] = sg * a.wT[3 * (size_t)ed + d];
    }
}

// wT[3 e + d] = wbar[d][e]: one 24-byte record per edge for the tets' gathers
__global__ __launch_bounds__(256) void k_interleave_w(TetArrays a)
{
    const int e = (int)blockIdx.x * 256 + (int)threadIdx.x;
    if (e >= a.E) return;
#pragma unroll
    for (int d = 0; d < 3; ++d) a.wT[3 * (size_t)e + d] = a.w[d][e];
}

// the share of x-bar of tet t at its local vertex v: 3 doubles at the
// (tet, vertex) pair's slot in the node-major list n2t
__device__ __forceinline__ void put_shares(const TetArrays &a, int t, const double (&xb)[4][3])
{
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        double *rec = a.scratch + (size_t)3 * a.n2t_pos[4 * t + v];
#pragma unroll
        for (int d = 0; d < 3; ++d) rec[d] = xb[v][d];
    }
}

__global__ __launch_bounds__(256) void k_tet_reverse(int T, TetArrays a, double period)
{
    const int t = (int)blockIdx.x * 256 + (int)threadIdx.x;
    if (t >= T) return;
    int g[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) g[v] = a.t2n[4 * t + v];
    double x[4][3], xb[4][3], cb[6][3];
    tet_x(a, g, period, x);
    tet_wbar(a, t, cb);
    tet_shares(x, cb, a.vol[g[0]] + a.vol[g[1]] + a.vol[g[2]] + a.vol[g[3]], xb);
    put_shares(a, t, xb);
}

// xbar[i] += sum over the tets around i of their share at i: one contiguous
// run of records per node
__global__ __launch_bounds__(256) void k_node_sum_xbar(TetArrays a)
{
    const int i = (int)blockIdx.x * 256 + (int)threadIdx.x;
    if (i >= a.N) return;
    double acc[3] = {0.0, 0.0, 0.0};
    const int end = a.n2t_off[i + 1];
    for (int j = a.n2t_off[i]; j < end; j += kSumAhead) {
        double r[kSumAhead][3];
#pragma unroll
        for (int u = 0; u < kSumAhead; ++u) {
            const double *rec = a.scratch + (size_t)3 * (j + u < end ? j + u : j);
#pragma unroll
            for (int d = 0; d < 3; ++d) r[u][d] = rec[d];
        }
#pragma unroll
        for (int u = 0; u < kSumAhead; ++u)
#pragma unroll
            for (int d = 0; d < 3; ++d)
                if (j + u < end) acc[d] += r[u][d];
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) a.xbar[d][i] += acc[d];
}

// ------------------------------------------------------------ ring form -- */
//
// The forward gather without per-tet records.  One workgroup per chunk of KG
// consecutive nodes stages the coordinates of its nodes and of its halo (the
// other vertices of the tets around its edges) in LDS; then one thread per
// edge of the chunk walks the tets around its edge in list order.  Around edge
// (a, b), tet (a, b, r, s) gives the face (x_r + x_s - x_a - x_b) x (x_s - x_r)
// / 24 (the formula above with p = a, q = b) and the determinant
// (x_b - x_a) . ((x_r - x_a) x (x_s - x_a)), six times the tet's volume; every
// difference is taken from x_a (wrapped to its nearest image in a periodic
// box).  The edge's weight gets the sum of its faces, and the sum of its
// determinants goes to edge_det; a node's volume is then the sum over its
// edges of edge_det / 72: a tet lies around three of its edges at each vertex,
// and each vertex owns a quarter of its volume.  Fixed orders throughout: the
// same bits on every run.

__device__ __forceinline__ void geo_diff(const double *x, const double *a, bool wrap, double period,
                                         double ip, double *d)
{
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        d[k] = x[k] - a[k];
        if (wrap) d[k] -= period * rint(d[k] * ip);
    }
}

// LDS rows: plane of (x, y) pairs, then plane of z (L rows each).
__device__ __forceinline__ void geo_get(const double *X, int L, uint32_t l, double *x)
{
    const double2 xy = reinterpret_cast<const double2 *>(X)[l];
    x[0] = xy.x;
    x[1] = xy.y;
    x[2] = X[2 * L + l];
}

// The edges of a chunk go in batches of kGeoThreads, one per thread; each
// batch's ring entries (one contiguous run) are first copied to LDS by the
// whole workgroup, so that the walks read LDS only.  Around edge (a, b) with
// chain c_0 .. c_k and d_i = x_(c_i) - x_a, tet i contributes
// (d_(i-1) + d_i - d_b) x (d_i - d_(i-1)) / 24 = (2 d_(i-1) x d_i
// - d_b x (d_i - d_(i-1))) / 24 to the face and d_b . (d_(i-1) x d_i) to the
// determinant sum; summed over the chain, the d_b terms telescope to
// d_b x (d_k - d_0), zero on a closed ring.  One vertex and one cross product
// per tet.
__global__ __launch_bounds__(kGeoThreads) void k_geo_rings(TetArrays a, double period)
{
    extern __shared__ __align__(16) unsigned char smem[];
    double *X = reinterpret_cast<double *>(smem);
    uint32_t *R32 = reinterpret_cast<uint32_t *>(smem + (size_t)a.L * 24);
    const uint16_t *R16 = reinterpret_cast<const uint16_t *>(R32);
    const uint32_t *ring32 = reinterpret_cast<const uint32_t *>(a.ring);
    const int L = a.L, KG = a.KG, c = (int)blockIdx.x, t = (int)threadIdx.x;
    const int v0 = c * KG, nown = min(KG, a.N - v0);
    const int h0 = a.halo_off[c], nh = a.halo_off[c + 1] - h0;
    const int2 ce = a.chunk_e[c];
    // the words of a batch: whole 4-byte words covering its entries, kGeoPre
    // per thread at most; the next batch's are loaded while this one computes
    uint32_t pre[kGeoPre];
    auto fetch = [&](int b0, int &q0, int &nq) {
        const int eb = ce.x + b0, nb = min(kGeoThreads, ce.y - b0);
        const int wb = a.ring_off[eb], we = a.ring_off[eb + nb];
        q0 = wb >> 1;
        nq = ((we + 1) >> 1) - q0;
#pragma unroll
        for (int u = 0; u < kGeoPre; ++u) {
            const int j = t + u * kGeoThreads;
            if (j < nq) pre[u] = ring32[q0 + j];
        }
    };
    int q0 = 0, nq = 0;
    if (ce.y > 0) fetch(0, q0, nq);
    for (int l = t; l < nown + nh; l += kGeoThreads) {
        const bool own = l < nown;
        const int g = own ? v0 + l : a.halo[h0 + l - nown];
        const int row = own ? l : KG + l - nown;
        reinterpret_cast<double2 *>(X)[row] = make_double2(a.x[0][g], a.x[1][g]);
        X[2 * L + row] = a.x[2][g];
    }
    const bool wrap = period > 0.0;
    const double ip = wrap ? 1.0 / period : 0.0;
    for (int b0 = 0; b0 < ce.y; b0 += kGeoThreads) {
        const int nb = min(kGeoThreads, ce.y - b0), eb = ce.x + b0;
        const int sh = 2 * q0;  // entry o of this batch sits at R16[o - sh]
        const bool act = t < nb;
        const int e = eb + t;
        int o0 = 0, o1 = 0;
        double w0[3] = {0.0, 0.0, 0.0};
        if (act) {
            o0 = a.ring_off[e] - sh;
            o1 = a.ring_off[e + 1] - sh;
            if (!a.write_w)
#pragma unroll
                for (int d = 0; d < 3; ++d) w0[d] = a.w[d][e];
        }
        __syncthreads();  // coordinates staged; the last batch's entries read
#pragma unroll
        for (int u = 0; u < kGeoPre; ++u) {
            const int j = t + u * kGeoThreads;
            if (j < nq) R32[j] = pre[u];
        }
        __syncthreads();
        if (b0 + kGeoThreads < ce.y) fetch(b0 + kGeoThreads, q0, nq);
        if (!act) continue;
        double xa[3], xb[3], db[3], d0[3], dp[3];
        geo_get(X, L, R16[o0], xa);
        geo_get(X, L, R16[o0 + 1], xb);
        geo_diff(xb, xa, wrap, period, ip, db);
        geo_get(X, L, R16[o0 + 2], d0);
        geo_diff(d0, xa, wrap, period, ip, d0);
#pragma unroll
        for (int d = 0; d < 3; ++d) dp[d] = d0[d];
        double C[3] = {0.0, 0.0, 0.0};
        for (int j = o0 + 3; j < o1; ++j) {
            double xn[3], dn[3], cr[3];
            geo_get(X, L, R16[j], xn);
            geo_diff(xn, xa, wrap, period, ip, dn);
            cross3(dp, dn, cr);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                C[d] += cr[d];
                dp[d] = dn[d];
            }
        }
        double ds[3], corr[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) ds[d] = dp[d] - d0[d];
        cross3(db, ds, corr);
#pragma unroll
        for (int d = 0; d < 3; ++d) a.w[d][e] = w0[d] + (2.0 * C[d] - corr[d]) * (1.0 / 24.0);
        a.edge_det[e] = db[0] * C[0] + db[1] * C[1] + db[2] * C[2];
    }
}

// Volumes, one workgroup per chunk: the determinant sums of the edges at its
// nodes go to LDS (its own edge range, coalesced, then the edges it shares
// with lower chunks, vsec), and each node adds those of its edges in the
// order of its slot list vloc: vol (+)= sum / 72.
__global__ __launch_bounds__(kGeoVolThreads) void k_geo_vol(TetArrays a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    double *D = reinterpret_cast<double *>(smem);
    const int c = (int)blockIdx.x, t = (int)threadIdx.x;
    const int v0 = c * a.KG, nown = min(a.KG, a.N - v0);
    const int2 ce = a.chunk_e[c];
    const int s0 = a.vsec_off[c], ns = a.vsec_off[c + 1] - s0;
    for (int j = t; j < ce.y; j += kGeoVolThreads) D[j] = a.edge_det[ce.x + j];
    for (int j = t; j < ns; j += kGeoVolThreads) D[ce.y + j] = a.edge_det[a.vsec[s0 + j]];
    __syncthreads();
    for (int l = t; l < nown; l += kGeoVolThreads) {
        const int i = v0 + l;
        const double vi = a.write_vol ? 0.0 : a.vol[i];
        double acc = 0.0;
        const int end = a.vloc_off[i + 1];
        for (int j = a.vloc_off[i]; j < end; ++j) acc += D[a.vloc[j]];
        a.vol[i] = vi + acc * (1.0 / 72.0);
    }
}

}  // namespace

int launch_geometry(bool adjoint, bool gather, int T, const TetArrays &a, double period,
                    hipStream_t st)
{
    if (T <= 0) return 0;
    if (gather) {
        const dim3 gt((T + 255) / 256), ge((a.E + 255) / 256), gn((a.N + 255) / 256);
        if (adjoint) {
            hipLaunchKernelGGL(k_interleave_w, ge, dim3(256), 0, st, a);
            hipLaunchKernelGGL(k_tet_reverse, gt, dim3(256), 0, st, T, a, period);
            hipLaunchKernelGGL(k_node_sum_xbar, gn, dim3(256), 0, st, a);
        } else if (a.ring) {
            const size_t lds = geo_ring_lds(a.L, a.RB);
            if (lds > 65536) {
                const hipError_t e = hipFuncSetAttribute(
                    reinterpret_cast<const void *>(k_geo_rings),
                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
                if (e != hipSuccess) return (int)e;
            }
            hipLaunchKernelGGL(k_geo_rings, dim3(a.nchunk), dim3(kGeoThreads), lds, st, a, period);
            hipLaunchKernelGGL(k_geo_vol, dim3(a.nchunk), dim3(kGeoVolThreads),
                               (size_t)a.DV * sizeof(double), st, a);
        } else {
            hipLaunchKernelGGL(k_tet_forward, gt, dim3(256), 0, st, T, a, period);
            hipLaunchKernelGGL(k_edge_sum_faces, ge, dim3(256), 0, st, a);
            hipLaunchKernelGGL(k_node_sum_vol, gn, dim3(256), 0, st, T, a);
        }
        return (int)hipGetLastError();
    }
    const int grid = (T + 255) / 256;
    if (adjoint)
        hipLaunchKernelGGL(k_geometry_adj, dim3(grid), dim3(256), 0, st, T, a, period);
    else
        hipLaunchKernelGGL(k_geometry, dim3(grid), dim3(256), 0, st, T, a, period);
    return (int)hipGetLastError();
}

}  // namespace gpu
}  // namespace opf
