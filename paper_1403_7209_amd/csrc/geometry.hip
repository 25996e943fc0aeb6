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
// atomics.  Gather: one thread per tet writes those results to a scratch
// buffer, then one thread per edge or node sums its incident tets' entries in
// a fixed order: no atomics, the same bits on every run.  The loop runs once
// per mesh (or once per design step for the reverse).
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
        const double sg = orient(a.e2n, a.t2e[6 * t + k], g[p]) * (1.0 / 24.0);
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
    for (int d = 0; d < 3; ++d) a.w[d][e] += acc[d];
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
    a.vol[i] += acc;
}

// record of tet t (12 doubles at t * 12): its share of x-bar at local vertex v
// at 3v + d
__global__ __launch_bounds__(256) void k_tet_reverse(int T, TetArrays a, double period)
{
    const int t = (int)blockIdx.x * 256 + (int)threadIdx.x;
    if (t >= T) return;
    int g[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) g[v] = a.t2n[4 * t + v];
    double x[4][3], xb[4][3];
    tet_x(a, g, period, x);
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int d = 0; d < 3; ++d) xb[v][d] = 0.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int p = kTetEdge[k][0], q = kTetEdge[k][1], r = kTetEdge[k][2], s = kTetEdge[k][3];
        const int ed = a.t2e[6 * t + k];
        const double sg = orient(a.e2n, ed, g[p]) * (1.0 / 24.0);
        double u[3], v[3], cb[3], ub[3], vb[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            u[d] = x[r][d] + x[s][d] - x[p][d] - x[q][d];
            v[d] = x[s][d] - x[r][d];
            cb[d] = sg * a.w[d][ed];
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
        for (int d = 0; d < 3; ++d) a.scratch[(size_t)t * 12 + 3 * v + d] = xb[v][d];
}

// xbar[i] += sum over the tets around i of their share at i
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
            const int tv = a.n2t[j + u < end ? j + u : j];
            const double *rec = a.scratch + (size_t)(tv >> 2) * 12 + 3 * (tv & 3);
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

}  // namespace

int launch_geometry(bool adjoint, bool gather, int T, const TetArrays &a, double period,
                    hipStream_t st)
{
    if (T <= 0) return 0;
    if (gather) {
        const dim3 gt((T + 255) / 256), ge((a.E + 255) / 256), gn((a.N + 255) / 256);
        if (adjoint) {
            hipLaunchKernelGGL(k_tet_reverse, gt, dim3(256), 0, st, T, a, period);
            hipLaunchKernelGGL(k_node_sum_xbar, gn, dim3(256), 0, st, a);
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
