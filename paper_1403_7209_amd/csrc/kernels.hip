// kernels.hip -- gfx950 kernels of the edge-flux path.
//
// Edge loops (Sec. 3.1 op_par_loop over edges with two OP_READ node arguments
// through the edge->node map, one direct weight and two OP_INC node
// increments) come in two forms:
//   * coloured: one workgroup per mini-partition, one launch per partition
//     colour (Sec. 4.1).  The partition's distinct nodes are staged into LDS
//     (the Sec. 4.1.2 staging, affordable with 160 KB of LDS per CU), every
//     thread evaluates its edges into registers, increments go into an LDS
//     accumulator one edge colour at a time, and the partition then adds its
//     accumulator to HBM with plain read-modify-write (partitions of one colour
//     share no node).  Deterministic.
//   * atomic: one thread per edge, FP64 atomic adds straight to HBM.
// Data are SoA (Sec. 4.1.2); every component is its own coalesced stream.
// The direct explicit stage and its residual norm are one grid-stride pass
// with a wavefront + LDS reduction per workgroup and a fixed-order second
// pass over the per-workgroup partial sums.
#include "kernels.hpp"

namespace opf {
namespace gpu {
namespace {

enum Mode { ANTI = 0, SAME = 1, GEN = 2 };

__device__ __forceinline__ double tsqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float tsqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double tabs(double x) { return fabs(x); }
__device__ __forceinline__ float tabs(float x) { return fabsf(x); }

template <typename T>
struct Prim {
    T u0, u1, u2, p, c, U;
};

// Velocity, pressure (ideal gas), sound speed and normal velocity of a node.
template <typename T>
__device__ __forceinline__ void prim(const T *q, const T *n, T gamma, Prim<T> &s)
{
    const T ir = T(1) / q[0];
    s.u0 = q[1] * ir;
    s.u1 = q[2] * ir;
    s.u2 = q[3] * ir;
    s.p = (gamma - T(1)) * (q[4] - T(0.5) * (q[1] * s.u0 + q[2] * s.u1 + q[3] * s.u2));
    s.c = tsqrt(gamma * s.p * ir);
    s.U = s.u0 * n[0] + s.u1 * n[1] + s.u2 * n[2];
}

// F = 1/2 (f(q_i) + f(q_j)).n - 1/2 lambda (q_j - q_i),
// lambda = |1/2 (U_i + U_j)| + 1/2 (c_i + c_j) |n|; +F to node i, -F to node j.
struct OpFlux {
    static constexpr int NIN = 6, NOUT = 6, NWOUT = 0, MODE = ANTI;
    template <typename T>
    __device__ static __forceinline__ void edge(const T *qi, const T *qj, const T *n, T gamma,
                                                double *yi, double *, double *)
    {
        Prim<T> a, b;
        prim(qi, n, gamma, a);
        prim(qj, n, gamma, b);
        const T h = T(0.5);
        const T nn = tsqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        const T hl = h * (tabs(h * (a.U + b.U)) + h * (a.c + b.c) * nn);
        yi[0] = (double)(h * (qi[0] * a.U + qj[0] * b.U) - hl * (qj[0] - qi[0]));
        yi[1] = (double)(h * (qi[1] * a.U + a.p * n[0] + qj[1] * b.U + b.p * n[0]) - hl * (qj[1] - qi[1]));
        yi[2] = (double)(h * (qi[2] * a.U + a.p * n[1] + qj[2] * b.U + b.p * n[1]) - hl * (qj[2] - qi[2]));
        yi[3] = (double)(h * (qi[3] * a.U + a.p * n[2] + qj[3] * b.U + b.p * n[2]) - hl * (qj[3] - qi[3]));
        yi[4] = (double)(h * ((qi[4] + a.p) * a.U + (qj[4] + b.p) * b.U) - hl * (qj[4] - qi[4]));
        yi[5] = (double)(h * (qi[5] * a.U + qj[5] * b.U) - hl * (qj[5] - qi[5]));
    }
};

// lambda_e added to both end nodes (local time-step denominator).
struct OpSpecrad {
    static constexpr int NIN = 5, NOUT = 1, NWOUT = 0, MODE = SAME;
    template <typename T>
    __device__ static __forceinline__ void edge(const T *qi, const T *qj, const T *n, T gamma,
                                                double *yi, double *, double *)
    {
        Prim<T> a, b;
        prim(qi, n, gamma, a);
        prim(qj, n, gamma, b);
        const T h = T(0.5);
        const T nn = tsqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        yi[0] = (double)(tabs(h * (a.U + b.U)) + h * (a.c + b.c) * nn);
    }
};

// Reverse of one node's share of the flux: given fb = dL/df (= Fbar/2), Ub
// (from lambda), cb (from lambda), accumulate into qb and nb.
__device__ __forceinline__ void node_reverse(const double *q, const Prim<double> &s,
                                             const double *n, double gamma, const double *fb,
                                             double Ub, double cb, double *qb, double *nb)
{
    // f = (q0 U, q1 U + p n0, q2 U + p n1, q3 U + p n2, (q4 + p) U, q5 U)
    Ub += fb[0] * q[0] + fb[1] * q[1] + fb[2] * q[2] + fb[3] * q[3] + fb[4] * (q[4] + s.p) +
          fb[5] * q[5];
    qb[0] += fb[0] * s.U;
    qb[1] += fb[1] * s.U;
    qb[2] += fb[2] * s.U;
    qb[3] += fb[3] * s.U;
    qb[4] += fb[4] * s.U;
    qb[5] += fb[5] * s.U;
    double pb = fb[1] * n[0] + fb[2] * n[1] + fb[3] * n[2] + fb[4] * s.U;
    nb[0] += fb[1] * s.p + Ub * s.u0;
    nb[1] += fb[2] * s.p + Ub * s.u1;
    nb[2] += fb[3] * s.p + Ub * s.u2;
    // U = u.n
    double ub0 = Ub * n[0], ub1 = Ub * n[1], ub2 = Ub * n[2];
    // c = sqrt(gamma p / rho)
    const double ir = 1.0 / q[0];
    const double sb = cb / (2.0 * s.c);
    pb += sb * gamma * ir;
    double rb = -sb * (s.c * s.c) * ir;
    // p = (gamma - 1)(q4 - ke/2), ke = q1 u0 + q2 u1 + q3 u2
    qb[4] += (gamma - 1.0) * pb;
    const double keb = -0.5 * (gamma - 1.0) * pb;
    qb[1] += keb * s.u0;
    qb[2] += keb * s.u1;
    qb[3] += keb * s.u2;
    ub0 += keb * q[1];
    ub1 += keb * q[2];
    ub2 += keb * q[3];
    // u_d = q_{1+d} / rho
    qb[1] += ub0 * ir;
    qb[2] += ub1 * ir;
    qb[3] += ub2 * ir;
    rb -= (ub0 * s.u0 + ub1 * s.u1 + ub2 * s.u2) * ir;
    qb[0] += rb;
}

// Reverse (adjoint) edge: inputs x = (q[6], rbar[6]) per node; with
// Fbar = rbar_i - rbar_j it returns qbar_i, qbar_j and nbar (direct).
// Forward intermediates are recomputed, never stored.
struct OpAdjoint {
    static constexpr int NIN = 12, NOUT = 6, NWOUT = 3, MODE = GEN;
    template <typename T>
    __device__ static __forceinline__ void edge(const T *xi, const T *xj, const T *n, T gamma,
                                                double *yi, double *yj, double *wo)
    {
        const double *qi = xi, *qj = xj;
        double Fb[6];
#pragma unroll
        for (int v = 0; v < 6; ++v) Fb[v] = xi[6 + v] - xj[6 + v];
        Prim<double> a, b;
        prim(qi, n, gamma, a);
        prim(qj, n, gamma, b);
        const double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        const double A = 0.5 * (a.U + b.U);
        const double lam = fabs(A) + 0.5 * (a.c + b.c) * nn;
        // F_v = (f_i,v + f_j,v)/2 - lam/2 (q_j,v - q_i,v)
        double lamb = 0.0;
#pragma unroll
        for (int v = 0; v < 6; ++v) {
            lamb += Fb[v] * (qj[v] - qi[v]);
            yi[v] = 0.5 * lam * Fb[v];
            yj[v] = -0.5 * lam * Fb[v];
        }
        lamb *= -0.5;
        const double Ab = (signbit(A) ? -1.0 : 1.0) * lamb;
        const double cb = 0.5 * nn * lamb;
        const double nnb = 0.5 * (a.c + b.c) * lamb;
        wo[0] = nnb * n[0] / nn;
        wo[1] = nnb * n[1] / nn;
        wo[2] = nnb * n[2] / nn;
        double fb[6];
#pragma unroll
        for (int v = 0; v < 6; ++v) fb[v] = 0.5 * Fb[v];
        node_reverse(qi, a, n, gamma, fb, 0.5 * Ab, cb, yi, wo);
        node_reverse(qj, b, n, gamma, fb, 0.5 * Ab, cb, yj, wo);
    }
};

struct PlanPtrs {
    const int *block_off;
    const int *uniq_off;
    const int *uniq;
    const uint32_t *lidx;
    const uint8_t *ecol;
    const int *block_ncol;
    const int *colour_blocks;
    int umax;
};

template <typename T>
struct Arrays {
    const T *x[12];
    double *y[6];
    const T *w[3];
    double *wo[3];
};

template <typename T>
Arrays<T> typed(const EdgeArrays &a)
{
    Arrays<T> r;
    for (int k = 0; k < 12; ++k) r.x[k] = static_cast<const T *>(a.xin[k]);
    for (int k = 0; k < 6; ++k) r.y[k] = a.yout[k];
    for (int k = 0; k < 3; ++k) r.w[k] = static_cast<const T *>(a.w[k]);
    for (int k = 0; k < 3; ++k) r.wo[k] = a.wout[k];
    return r;
}

// Maps workgroup k of n so that XCD (k mod 8) receives one contiguous range:
// workgroups are dispatched round-robin over the 8 XCDs, each with its own L2.
__device__ __forceinline__ int xcd_map(int k, int n)
{
    const int x = k & 7, i = k >> 3, per = n >> 3, rem = n & 7;
    return x * per + min(x, rem) + i;
}

template <typename T, class Op>
__host__ __device__ constexpr size_t lds_x_bytes(int umax)
{
    return ((size_t)Op::NIN * umax * sizeof(T) + 15) & ~(size_t)15;
}

template <typename T, class Op>
constexpr size_t lds_bytes(int umax)
{
    return lds_x_bytes<T, Op>(umax) + (size_t)Op::NOUT * umax * sizeof(double);
}

template <typename T, class Op, int NT, int EPT>
__global__ __launch_bounds__(NT) void k_edge_lds(PlanPtrs p, Arrays<T> a, T gamma, int cbase,
                                                 int ncb, int remap)
{
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NY = Op::MODE == GEN ? 2 * Op::NOUT : Op::NOUT;
    const int umax = p.umax;
    T *sx = reinterpret_cast<T *>(smem);
    double *sy = reinterpret_cast<double *>(smem + lds_x_bytes<T, Op>(umax));

    const int k = remap ? xcd_map((int)blockIdx.x, ncb) : (int)blockIdx.x;
    const int b = p.colour_blocks[cbase + k];
    const int e0 = p.block_off[b], ne = p.block_off[b + 1] - e0;
    const int u0 = p.uniq_off[b], nu = p.uniq_off[b + 1] - u0;

    // stage the partition's node data, clear its accumulator
    for (int u = threadIdx.x; u < nu; u += NT) {
        const int g = p.uniq[u0 + u];
#pragma unroll
        for (int v = 0; v < Op::NIN; ++v) sx[v * umax + u] = a.x[v][g];
#pragma unroll
        for (int v = 0; v < Op::NOUT; ++v) sy[v * umax + u] = 0.0;
    }
    __syncthreads();

    double y[EPT][NY];
    int li[EPT], lj[EPT], col[EPT];
#pragma unroll
    for (int t = 0; t < EPT; ++t) {
        const int e = threadIdx.x + t * NT;
        col[t] = -1;
        li[t] = lj[t] = 0;
        if (e < ne) {
            const uint32_t l = p.lidx[e0 + e];
            li[t] = (int)(l & 0xffffu);
            lj[t] = (int)(l >> 16);
            col[t] = p.ecol[e0 + e];
            T xi[Op::NIN], xj[Op::NIN], n[3];
#pragma unroll
            for (int v = 0; v < Op::NIN; ++v) {
                xi[v] = sx[v * umax + li[t]];
                xj[v] = sx[v * umax + lj[t]];
            }
#pragma unroll
            for (int d = 0; d < 3; ++d) n[d] = a.w[d][e0 + e];
            double wo[3] = {0.0, 0.0, 0.0};
            Op::edge(xi, xj, n, gamma, y[t], y[t] + Op::NOUT, wo);
            if (Op::NWOUT) {
#pragma unroll
                for (int d = 0; d < 3; ++d) a.wo[d][e0 + e] = wo[d];
            }
        }
    }

    // increments, one edge colour at a time (same-colour edges share no node)
    const int ncol = p.block_ncol[b];
    for (int c = 0; c < ncol; ++c) {
#pragma unroll
        for (int t = 0; t < EPT; ++t) {
            if (col[t] == c) {
#pragma unroll
                for (int v = 0; v < Op::NOUT; ++v) {
                    const double yi = y[t][v];
                    const double yj = Op::MODE == ANTI ? -yi : Op::MODE == SAME ? yi : y[t][Op::NOUT + v];
                    sy[v * umax + li[t]] += yi;
                    sy[v * umax + lj[t]] += yj;
                }
            }
        }
        __syncthreads();
    }

    // add the partition's accumulator to HBM (no other partition of this
    // colour touches these nodes)
    for (int u = threadIdx.x; u < nu; u += NT) {
        const int g = p.uniq[u0 + u];
#pragma unroll
        for (int v = 0; v < Op::NOUT; ++v) a.y[v][g] += sy[v * umax + u];
    }
}

template <typename T, class Op>
__global__ __launch_bounds__(256) void k_edge_atomic(const int2 *__restrict__ e2n, int E,
                                                     Arrays<T> a, T gamma, int remap)
{
    const int blk = remap ? xcd_map((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x;
    const int e = blk * 256 + (int)threadIdx.x;
    if (e >= E) return;
    const int2 ij = e2n[e];
    T xi[Op::NIN], xj[Op::NIN], n[3];
#pragma unroll
    for (int v = 0; v < Op::NIN; ++v) {
        xi[v] = a.x[v][ij.x];
        xj[v] = a.x[v][ij.y];
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) n[d] = a.w[d][e];
    constexpr int NY = Op::MODE == GEN ? 2 * Op::NOUT : Op::NOUT;
    double y[NY];
    double wo[3] = {0.0, 0.0, 0.0};
    Op::edge(xi, xj, n, gamma, y, y + Op::NOUT, wo);
#pragma unroll
    for (int v = 0; v < Op::NOUT; ++v) {
        const double yi = y[v];
        const double yj = Op::MODE == ANTI ? -yi : Op::MODE == SAME ? yi : y[Op::NOUT + v];
        unsafeAtomicAdd(a.y[v] + ij.x, yi);
        unsafeAtomicAdd(a.y[v] + ij.y, yj);
    }
    if (Op::NWOUT) {
#pragma unroll
        for (int d = 0; d < 3; ++d) a.wo[d][e] = wo[d];
    }
}

// ------------------------------------------------------ reductions -- */

template <int NV>
__device__ __forceinline__ void block_sum(double (&acc)[NV], double *out)
{
    __shared__ double red[4][NV];
#pragma unroll
    for (int v = 0; v < NV; ++v)
        for (int off = 32; off > 0; off >>= 1) acc[v] += __shfl_down(acc[v], off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int v = 0; v < NV; ++v) red[wave][v] = acc[v];
    __syncthreads();
    if (threadIdx.x < NV) {
        const int v = threadIdx.x;
        out[v] = ((red[0][v] + red[1][v]) + red[2][v]) + red[3][v];
    }
}

template <typename T>
struct RkPtrs {
    const T *q0[6];
    double *res[6];
    const double *vol;
    T *q[6];
};

template <typename T>
__global__ __launch_bounds__(kRkThreads) void k_rk_stage(int N, RkPtrs<T> a, double alpha_dt,
                                                         double *partial)
{
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const int stride = (int)gridDim.x * kRkThreads;
    for (int i = (int)blockIdx.x * kRkThreads + (int)threadIdx.x; i < N; i += stride) {
        const double vi = a.vol[i];
#pragma unroll
        for (int v = 0; v < 6; ++v) {
            const double r = a.res[v][i];
            acc[v] += r * r;
            a.q[v][i] = (T)((double)a.q0[v][i] - alpha_dt * r / vi);
            a.res[v][i] = 0.0;
        }
    }
    block_sum<6>(acc, partial + 6 * blockIdx.x);
}

__global__ __launch_bounds__(256) void k_sum_partials(int nparts, const double *partial,
                                                      double *ss)
{
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int k = threadIdx.x; k < nparts; k += 256)
#pragma unroll
        for (int v = 0; v < 6; ++v) acc[v] += partial[6 * k + v];
    __shared__ double tot[6];
    block_sum<6>(acc, tot);
    __syncthreads();
    if (threadIdx.x < 6) ss[threadIdx.x] += tot[threadIdx.x];
}

template <int NV>
__device__ __forceinline__ void block_min(double (&m)[NV], double *out)
{
    __shared__ double red[4][NV];
#pragma unroll
    for (int v = 0; v < NV; ++v)
        for (int off = 32; off > 0; off >>= 1) m[v] = fmin(m[v], __shfl_down(m[v], off, 64));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int v = 0; v < NV; ++v) red[wave][v] = m[v];
    __syncthreads();
    if (threadIdx.x < NV) {
        const int v = threadIdx.x;
        out[v] = fmin(fmin(red[0][v], red[1][v]), fmin(red[2][v], red[3][v]));
    }
}

__global__ __launch_bounds__(kRkThreads) void k_dt_min(int N, const double *vol,
                                                       const double *lam, double *partial)
{
    double m[1] = {INFINITY};
    const int stride = (int)gridDim.x * kRkThreads;
    for (int i = (int)blockIdx.x * kRkThreads + (int)threadIdx.x; i < N; i += stride)
        m[0] = fmin(m[0], vol[i] / lam[i]);
    block_min<1>(m, partial + blockIdx.x);
}

__global__ __launch_bounds__(256) void k_min_partials(int nparts, const double *partial,
                                                      double cfl, double *dt)
{
    double m[1] = {INFINITY};
    for (int k = threadIdx.x; k < nparts; k += 256) m[0] = fmin(m[0], partial[k]);
    __shared__ double tot[1];
    block_min<1>(m, tot);
    __syncthreads();
    if (threadIdx.x == 0) dt[0] = fmin(dt[0], cfl * tot[0]);
}

// ----------------------------------------------------------- launchers -- */

PlanPtrs plan_ptrs(const DevPlan &P)
{
    return PlanPtrs{P.block_off, P.uniq_off, P.uniq, P.lidx, P.ecol, P.block_ncol,
                    P.colour_blocks, P.umax};
}

template <typename T, class Op, int NT, int EPT>
int run_lds(const DevPlan &P, const EdgeArrays &a, double gamma, hipStream_t st,
            const LaunchOpts &lo)
{
    const size_t lds = lds_bytes<T, Op>(P.umax);
    const Arrays<T> ta = typed<T>(a);
    const PlanPtrs pp = plan_ptrs(P);
    for (int c = 0; c < P.nc; ++c) {
        const int n = P.colour_off[c + 1] - P.colour_off[c];
        if (n <= 0) continue;
        hipLaunchKernelGGL((k_edge_lds<T, Op, NT, EPT>), dim3(n), dim3(NT), lds, st, pp, ta,
                           (T)gamma, P.colour_off[c], n, lo.xcd_remap);
    }
    return (int)hipGetLastError();
}

template <typename T, class Op>
int run_lds_bs(const DevPlan &P, const EdgeArrays &a, double gamma, hipStream_t st,
               const LaunchOpts &lo)
{
    switch (P.block_size) {
    case 64: return run_lds<T, Op, 64, 1>(P, a, gamma, st, lo);
    case 128: return run_lds<T, Op, 128, 1>(P, a, gamma, st, lo);
    case 256: return run_lds<T, Op, 256, 1>(P, a, gamma, st, lo);
    case 512: return run_lds<T, Op, 256, 2>(P, a, gamma, st, lo);
    case 1024: return run_lds<T, Op, 256, 4>(P, a, gamma, st, lo);
    case 2048: return run_lds<T, Op, 256, 8>(P, a, gamma, st, lo);
    default: return (int)hipErrorInvalidValue;
    }
}

template <typename T, class Op>
int run_atomic(const DevPlan &P, const EdgeArrays &a, double gamma, hipStream_t st,
               const LaunchOpts &lo)
{
    if (P.E <= 0) return 0;
    const int grid = (P.E + 255) / 256;
    hipLaunchKernelGGL((k_edge_atomic<T, Op>), dim3(grid), dim3(256), 0, st, P.e2n, P.E,
                       typed<T>(a), (T)gamma, lo.xcd_remap);
    return (int)hipGetLastError();
}

template <typename T, class Op>
int run_edge(int variant, const DevPlan &P, const EdgeArrays &a, double gamma, hipStream_t st,
             const LaunchOpts &lo)
{
    return variant == 1 ? run_atomic<T, Op>(P, a, gamma, st, lo)
                        : run_lds_bs<T, Op>(P, a, gamma, st, lo);
}

template <typename T, class Op>
int raise_limits(size_t bytes)
{
    const void *fns[] = {
        reinterpret_cast<const void *>(&k_edge_lds<T, Op, 64, 1>),
        reinterpret_cast<const void *>(&k_edge_lds<T, Op, 128, 1>),
        reinterpret_cast<const void *>(&k_edge_lds<T, Op, 256, 1>),
        reinterpret_cast<const void *>(&k_edge_lds<T, Op, 256, 2>),
        reinterpret_cast<const void *>(&k_edge_lds<T, Op, 256, 4>),
        reinterpret_cast<const void *>(&k_edge_lds<T, Op, 256, 8>)};
    for (const void *f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return (int)e;
    }
    return 0;
}

}  // namespace

size_t edge_lds_bytes(int op, bool fp32, int umax)
{
    if (op == OP_ADJOINT) return lds_bytes<double, OpAdjoint>(umax);
    if (op == OP_SPECRAD)
        return fp32 ? lds_bytes<float, OpSpecrad>(umax) : lds_bytes<double, OpSpecrad>(umax);
    return fp32 ? lds_bytes<float, OpFlux>(umax) : lds_bytes<double, OpFlux>(umax);
}

int set_lds_limit(size_t bytes)
{
    int rc = 0;
    if (!rc) rc = raise_limits<double, OpFlux>(bytes);
    if (!rc) rc = raise_limits<float, OpFlux>(bytes);
    if (!rc) rc = raise_limits<double, OpSpecrad>(bytes);
    if (!rc) rc = raise_limits<float, OpSpecrad>(bytes);
    if (!rc) rc = raise_limits<double, OpAdjoint>(bytes);
    return rc;
}

int launch_edge(int op, bool fp32, int variant, const DevPlan &P, const EdgeArrays &a,
                double gamma, hipStream_t st, const LaunchOpts &lo)
{
    switch (op) {
    case OP_FLUX:
        return fp32 ? run_edge<float, OpFlux>(variant, P, a, gamma, st, lo)
                    : run_edge<double, OpFlux>(variant, P, a, gamma, st, lo);
    case OP_SPECRAD:
        return fp32 ? run_edge<float, OpSpecrad>(variant, P, a, gamma, st, lo)
                    : run_edge<double, OpSpecrad>(variant, P, a, gamma, st, lo);
    case OP_ADJOINT:
        if (fp32) return (int)hipErrorInvalidValue;
        return run_edge<double, OpAdjoint>(variant, P, a, gamma, st, lo);
    default: return (int)hipErrorInvalidValue;
    }
}

template <typename T>
static int run_rk(int N, const NodeArrays &a, double alpha_dt, double *ss, double *partial,
                  hipStream_t st)
{
    RkPtrs<T> p;
    for (int v = 0; v < 6; ++v) {
        p.q0[v] = static_cast<const T *>(a.q0[v]);
        p.res[v] = a.res[v];
        p.q[v] = static_cast<T *>(a.q[v]);
    }
    p.vol = a.vol;
    const int grid = std::min(kRkBlocks, std::max(1, (N + kRkThreads - 1) / kRkThreads));
    hipLaunchKernelGGL((k_rk_stage<T>), dim3(grid), dim3(kRkThreads), 0, st, N, p, alpha_dt,
                       partial);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, grid, partial, ss);
    return (int)hipGetLastError();
}

int launch_rk_stage(bool fp32, int N, const NodeArrays &a, double alpha_dt, double *ss,
                    double *partial, hipStream_t st)
{
    return fp32 ? run_rk<float>(N, a, alpha_dt, ss, partial, st)
                : run_rk<double>(N, a, alpha_dt, ss, partial, st);
}

int launch_dt_min(int N, const double *vol, const double *lam, double cfl, double *dt,
                  double *partial, hipStream_t st)
{
    const int grid = std::min(kRkBlocks, std::max(1, (N + kRkThreads - 1) / kRkThreads));
    hipLaunchKernelGGL(k_dt_min, dim3(grid), dim3(kRkThreads), 0, st, N, vol, lam, partial);
    hipLaunchKernelGGL(k_min_partials, dim3(1), dim3(256), 0, st, grid, partial, cfl, dt);
    return (int)hipGetLastError();
}

}  // namespace gpu
}  // namespace opf
