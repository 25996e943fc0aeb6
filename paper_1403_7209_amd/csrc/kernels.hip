// kernels.hip -- gfx950 kernels of the edge-flux path.
//
// An edge loop is an op_par_loop over edges (Sec. 3.1) with OP_READ node
// arguments through the edge->node map, one direct 3-vector weight and OP_INC
// node increments.  Every kernel first turns a node's inputs into a "staged"
// record once per node (state and primitives: velocity, sound speed; the
// flux rebuilds the pressure as rho c^2 / gamma), so the per-edge work needs
// no division or square root besides |n_e|.
// Four ways to resolve the increments:
//   * coloured (Sec. 4.1): one workgroup per mini-partition, one launch per
//     partition colour.  The partition's distinct nodes are staged in LDS (the
//     Sec. 4.1.2 staging; gfx950 has 160 KB of LDS per CU), increments go into
//     an LDS accumulator one edge colour at a time (or with LDS FP64 atomics in
//     the ablation variant), then the partition adds its accumulator to HBM
//     with plain read-modify-write: partitions of one colour share no node.
//   * atomic: one thread per edge, FP64 atomic adds straight to HBM.
//   * flat: one level of edge colours over the whole mesh, one launch per
//     colour, one thread per edge, plain read-add-write in HBM (the
//     single-level counterpart of the Sec. 4.1 plan).
//   * owner: one workgroup per contiguous cluster of K nodes runs every edge
//     that touches the cluster (edges joining two clusters run in both), adds
//     only into its own nodes' LDS accumulator (ds_add_f64) and writes each
//     node's residual exactly once, coalesced.  Single launch, no partition
//     colours, no HBM atomics -- the owner-compute rule of the paper's
//     distributed back-end (redundant execution of halo edges, Sec. 3.2 and
//     4.2) applied to the workgroups of one GPU.
// Data are SoA (Sec. 4.1.2): every component is its own coalesced stream.
// The direct stage update and its residual norm are one grid-stride pass
// with a wavefront + LDS reduction per workgroup and a fixed-order second
// pass over the per-workgroup partial sums; with the owner variant the update
// can instead run at the end of each owner workgroup (the fused stage), whose
// partial sums go through an LDS tree to the same second pass.
#include <algorithm>
#include <type_traits>

#include "kernels.hpp"

// Scratch of the fused stage for callers that cannot allocate: per-cluster
// partial sums (6 doubles per cluster).  Host code must not pass this name to a
// kernel -- on the host it is only a stand-in for the symbol; the device address
// comes from static_scratch_address(), resolved once per device.
static __device__ __align__(256) double scratch[opf::gpu::kSumTail + 6 * opf::gpu::kStaticMaxClusters];

// Tuning of the owner kernel per (type, op): edges each thread resolves before
// computing (B), and the waves per SIMD the register allocator must allow
// (0: no constraint).  Occupancy, not bandwidth per wave, limits these loops.
#ifndef OPF_FLUX64_BATCH
#define OPF_FLUX64_BATCH 2
#endif
#ifndef OPF_FLUX64_CUT_BATCH
#define OPF_FLUX64_CUT_BATCH 1
#endif
#ifndef OPF_FLUX64_WAVES
#define OPF_FLUX64_WAVES 6
#endif
#ifndef OPF_FLUX32_BATCH
#define OPF_FLUX32_BATCH 2
#endif
#ifndef OPF_FLUX32_CUT_BATCH
#define OPF_FLUX32_CUT_BATCH 2
#endif
#ifndef OPF_FLUX32_WAVES
#define OPF_FLUX32_WAVES 8
#endif
#ifndef OPF_ADJ_BATCH
#define OPF_ADJ_BATCH 1
#endif
#ifndef OPF_ADJ_CUT_BATCH
#define OPF_ADJ_CUT_BATCH 1
#endif
#ifndef OPF_ADJ_WAVES
#define OPF_ADJ_WAVES 4
#endif
#ifndef OPF_FLUX2_CUT_BATCH
#define OPF_FLUX2_CUT_BATCH 1
#endif
// The second-order loop holds 30 values per node in LDS: one workgroup per CU,
// so its workgroups take more threads (768: it spills registers at 1024).  The
// gradient runs in halves of 12 values per node, three 512-thread workgroups
// per CU.
#ifndef OPF_GRAD_BATCH
#define OPF_GRAD_BATCH 2
#endif
#ifndef OPF_GRAD_THREADS
#define OPF_GRAD_THREADS 512
#endif
#ifndef OPF_FLUX2_BATCH
#define OPF_FLUX2_BATCH 2
#endif
#ifndef OPF_FLUX2_THREADS
#define OPF_FLUX2_THREADS 768
#endif

namespace opf {
namespace gpu {
namespace {

enum Mode { ANTI = 0, SAME = 1, GEN = 2 };

// Reciprocal and square root from the hardware approximations (relative error
// about 2^-24).  FP64 refines each by one Newton (Goldschmidt) step, which
// squares the error: a few ulp, far inside the loop's tolerance, at a third of
// the instructions of the correctly rounded sequences.  FP32 uses them as they
// are (about 1 ulp).  Arguments are densities, squared sound speeds and squared
// face areas: non-negative; a zero square root comes out as 0.
__device__ __forceinline__ double trcp(double x)
{
    const double r = __builtin_amdgcn_rcp(x);
    return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ float trcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double tsqrt(double x)
{
    const double r = __builtin_amdgcn_rsq(fmax(x, 1e-300));
    const double g = x * r, h = 0.5 * r;
    return fma(g, fma(-g, h, 0.5), g);
}
__device__ __forceinline__ float tsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double tabs(double x) { return fabs(x); }
__device__ __forceinline__ float tabs(float x) { return fabsf(x); }
// x with its sign flipped when s is set (one XOR of the sign bit).
__device__ __forceinline__ double flip(double x, uint32_t s)
{
    return __hiloint2double(__double2hiint(x) ^ (int)(s << 31), __double2loint(x));
}
__device__ __forceinline__ float flip(float x, uint32_t s)
{
    return __uint_as_float(__float_as_uint(x) ^ (s << 31));
}

// ----------------------------------------------------------- edge math -- */

// F = 1/2 (f(q_i) + f(q_j)).n - 1/2 lambda (q_j - q_i),
// lambda = |1/2 (U_i + U_j)| + 1/2 (c_i + c_j) |n|, U = u.n; +F to node i,
// -F to node j.  Staged record: rho, u[0..2], rho E, rho phi, c (the
// momentum is rebuilt as rho u, the pressure as rho c^2 / gamma: seven values
// per node keep three FP64 owner workgroups within one CU's LDS).
struct OpFlux {
    static constexpr int NIN = 6, NS = 7, NOUT = 6, NW = 3, NWOUT = 0, MODE = ANTI;
    template <typename T>
    __device__ static __forceinline__ void stage(const T *x, T *s, T gamma)
    {
        const T ir = trcp(x[0]);
        s[0] = x[0];
        s[1] = x[1] * ir;
        s[2] = x[2] * ir;
        s[3] = x[3] * ir;
        s[4] = x[4];
        s[5] = x[5];
        const T p = (gamma - T(1)) * (x[4] - T(0.5) * (x[1] * s[1] + x[2] * s[2] + x[3] * s[3]));
        s[6] = tsqrt(gamma * p * ir);
    }
    template <typename T>
    __device__ static __forceinline__ void edge(const T *a, const T *b, const T *n, T gamma,
                                                double *yi, double *, double *)
    {
        const T h = T(0.5);
        const T Ua = a[1] * n[0] + a[2] * n[1] + a[3] * n[2];
        const T Ub = b[1] * n[0] + b[2] * n[1] + b[3] * n[2];
        const T nn = tsqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        const T hl = h * (tabs(h * (Ua + Ub)) + h * (a[6] + b[6]) * nn);
        const T ma = a[0] * Ua, mb = b[0] * Ub;  // mass fluxes
        const T ig = T(1) / gamma;
        const T pa = a[0] * a[6] * a[6] * ig, pb = b[0] * b[6] * b[6] * ig;
        const T pp = pa + pb;
        yi[0] = (double)(h * (ma + mb) - hl * (b[0] - a[0]));
        yi[1] = (double)(h * (ma * a[1] + mb * b[1] + pp * n[0]) - hl * (b[0] * b[1] - a[0] * a[1]));
        yi[2] = (double)(h * (ma * a[2] + mb * b[2] + pp * n[1]) - hl * (b[0] * b[2] - a[0] * a[2]));
        yi[3] = (double)(h * (ma * a[3] + mb * b[3] + pp * n[2]) - hl * (b[0] * b[3] - a[0] * a[3]));
        yi[4] = (double)(h * ((a[4] + pa) * Ua + (b[4] + pb) * Ub) - hl * (b[4] - a[4]));
        yi[5] = (double)(h * (a[5] * Ua + b[5] * Ub) - hl * (b[5] - a[5]));
    }
};

// lambda_e added to both end nodes (local time-step denominator).
// Staged record: u[0..2], c.
struct OpSpecrad {
    static constexpr int NIN = 5, NS = 4, NOUT = 1, NW = 3, NWOUT = 0, MODE = SAME;
    template <typename T>
    __device__ static __forceinline__ void stage(const T *x, T *s, T gamma)
    {
        const T ir = trcp(x[0]);
        s[0] = x[1] * ir;
        s[1] = x[2] * ir;
        s[2] = x[3] * ir;
        const T p = (gamma - T(1)) * (x[4] - T(0.5) * (x[1] * s[0] + x[2] * s[1] + x[3] * s[2]));
        s[3] = tsqrt(gamma * p * ir);
    }
    template <typename T>
    __device__ static __forceinline__ void edge(const T *a, const T *b, const T *n, T,
                                                double *yi, double *, double *)
    {
        const T h = T(0.5);
        const T Ua = a[0] * n[0] + a[1] * n[1] + a[2] * n[2];
        const T Ub = b[0] * n[0] + b[1] * n[1] + b[2] * n[2];
        const T nn = tsqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        yi[0] = (double)(tabs(h * (Ua + Ub)) + h * (a[3] + b[3]) * nn);
    }
};

template <typename T>
struct Prim {
    T u0, u1, u2, p, c, U;
};

template <typename T>
__device__ __forceinline__ void prim(const T *q, const T *n, T gamma, Prim<T> &s)
{
    const T ir = trcp(q[0]);
    s.u0 = q[1] * ir;
    s.u1 = q[2] * ir;
    s.u2 = q[3] * ir;
    s.p = (gamma - T(1)) * (q[4] - T(0.5) * (q[1] * s.u0 + q[2] * s.u1 + q[3] * s.u2));
    s.c = tsqrt(gamma * s.p * ir);
    s.U = s.u0 * n[0] + s.u1 * n[1] + s.u2 * n[2];
}

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
    const double ir = trcp(q[0]);
    const double sb = 0.5 * cb * trcp(s.c);
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

// Reverse (adjoint) edge: inputs (q[6], rbar[6]) per node; with
// Fbar = rbar_i - rbar_j it returns qbar_i, qbar_j and nbar (direct).
// Forward intermediates are recomputed, never stored.
struct OpAdjoint {
    static constexpr int NIN = 12, NS = 12, NOUT = 6, NW = 3, NWOUT = 3, MODE = GEN;
    template <typename T>
    __device__ static __forceinline__ void stage(const T *x, T *s, T)
    {
#pragma unroll
        for (int v = 0; v < 12; ++v) s[v] = x[v];
    }
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
        const double nn = tsqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
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
        const double inn = nnb * trcp(nn);
        wo[0] = inn * n[0];
        wo[1] = inn * n[1];
        wo[2] = inn * n[2];
        double fb[6];
#pragma unroll
        for (int v = 0; v < 6; ++v) fb[v] = 0.5 * Fb[v];
        node_reverse(qi, a, n, gamma, fb, 0.5 * Ab, cb, yi, wo);
        node_reverse(qj, b, n, gamma, fb, 0.5 * Ab, cb, yj, wo);
    }
};

// Green-Gauss sums: +1/2 (q_i + q_j) n_e into node i (component 3v + d),
// the negative into node j.  Staged record: the state itself.
struct OpGrad {
    static constexpr int NIN = 6, NS = 6, NOUT = 18, NW = 3, NWOUT = 0, MODE = ANTI;
    template <typename T>
    __device__ static __forceinline__ void stage(const T *x, T *s, T)
    {
#pragma unroll
        for (int v = 0; v < 6; ++v) s[v] = x[v];
    }
    template <typename T>
    __device__ static __forceinline__ void edge(const T *a, const T *b, const T *n, T,
                                                double *yi, double *, double *)
    {
#pragma unroll
        for (int v = 0; v < 6; ++v) {
            const T f = T(0.5) * (a[v] + b[v]);
#pragma unroll
            for (int d = 0; d < 3; ++d) yi[3 * v + d] = (double)(f * n[d]);
        }
    }
};

// The owner variant runs the Green-Gauss sums in two halves: three variables
// (9 sums) per workgroup, two workgroups per cluster, so that the 9 LDS sums
// per node leave room for three workgroups per CU where the 18 left room for
// one.  The kernel shifts the node inputs and outputs by the half it takes.
struct OpGradH {
    static constexpr int NIN = 3, NS = 3, NOUT = 9, NW = 3, NWOUT = 0, MODE = ANTI;
    template <typename T>
    __device__ static __forceinline__ void stage(const T *x, T *s, T)
    {
#pragma unroll
        for (int v = 0; v < 3; ++v) s[v] = x[v];
    }
    template <typename T>
    __device__ static __forceinline__ void edge(const T *a, const T *b, const T *n, T,
                                                double *yi, double *, double *)
    {
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            const T f = T(0.5) * (a[v] + b[v]);
#pragma unroll
            for (int d = 0; d < 3; ++d) yi[3 * v + d] = (double)(f * n[d]);
        }
    }
};

// Second-order flux: the OpFlux flux of the states reconstructed linearly to
// the edge midpoint.  Node inputs: q (6), Green-Gauss sums G (18), vol (1);
// staged record: q and the gradient G / vol.  Edge inputs: n, then dx = x_j - x_i.
struct OpFlux2 {
    static constexpr int NIN = 25, NS = 24, NOUT = 6, NW = 6, NWOUT = 0, MODE = ANTI;
    template <typename T>
    __device__ static __forceinline__ void stage(const T *x, T *s, T)
    {
        const T iv = trcp(x[24]);
#pragma unroll
        for (int v = 0; v < 6; ++v) s[v] = x[v];
#pragma unroll
        for (int k = 0; k < 18; ++k) s[6 + k] = x[6 + k] * iv;
    }
    template <typename T>
    __device__ static __forceinline__ void edge(const T *a, const T *b, const T *w, T gamma,
                                                double *yi, double *, double *)
    {
        const T h = T(0.5);
        T qL[6], qR[6];
#pragma unroll
        for (int v = 0; v < 6; ++v) {
            qL[v] = a[v] + h * (a[6 + 3 * v] * w[3] + a[7 + 3 * v] * w[4] + a[8 + 3 * v] * w[5]);
            qR[v] = b[v] - h * (b[6 + 3 * v] * w[3] + b[7 + 3 * v] * w[4] + b[8 + 3 * v] * w[5]);
        }
        T sL[OpFlux::NS], sR[OpFlux::NS];
        OpFlux::stage(qL, sL, gamma);
        OpFlux::stage(qR, sR, gamma);
        OpFlux::edge(sL, sR, w, gamma, yi, nullptr, nullptr);
    }
};

// B: edges each thread resolves before computing in the interior loop, BC in
// the cut-visit loop (whose gathered records cost registers).
// FOREIGN: the cut visits in the plan's foreign-node order (the lanes of a
// wavefront share foreign records: pays where those records are wide and
// bandwidth binds) rather than the bank-spread order (pays where the LDS
// updates bind).
// STREAM: non-temporal hints on the loop's once-touched data (ld1/st1) when
// its arrays exceed the last-level cache (owner_streams).  They pay in the
// flux loops (3-5 %) and cost in the adjoint, gradient and second-order loops
// (4-17 %), whose wider records or scattered edge writes do better through
// the normal cache policy.
template <typename T, class Op>
struct OwnerTune {
    static constexpr int B = 2, BC = 2, WAVES = 0, NT = kOwnerThreads;
    static constexpr bool FOREIGN = false, STREAM = false;
};
template <>
struct OwnerTune<float, OpFlux> {
    static constexpr int B = OPF_FLUX32_BATCH, BC = OPF_FLUX32_CUT_BATCH, WAVES = OPF_FLUX32_WAVES,
                         NT = kOwnerThreads;
    static constexpr bool FOREIGN = false, STREAM = true;
};
template <>
struct OwnerTune<double, OpFlux> {
    static constexpr int B = OPF_FLUX64_BATCH, BC = OPF_FLUX64_CUT_BATCH, WAVES = OPF_FLUX64_WAVES,
                         NT = kOwnerThreads;
    static constexpr bool FOREIGN = true, STREAM = true;
};
template <>
struct OwnerTune<double, OpAdjoint> {
    static constexpr int B = OPF_ADJ_BATCH, BC = OPF_ADJ_CUT_BATCH, WAVES = OPF_ADJ_WAVES,
                         NT = kOwnerThreads;
    static constexpr bool FOREIGN = true, STREAM = false;
};
template <>
struct OwnerTune<double, OpGradH> {
    static constexpr int B = OPF_GRAD_BATCH, BC = OPF_GRAD_BATCH, WAVES = 0, NT = OPF_GRAD_THREADS;
    static constexpr bool FOREIGN = false, STREAM = false;
};

// The op the owner variant runs for Op, and whether in two halves per cluster.
template <class Op>
struct OwnerOp {
    using type = Op;
    static constexpr bool HALVES = false;
};
template <>
struct OwnerOp<OpGrad> {
    using type = OpGradH;
    static constexpr bool HALVES = true;
};
template <>
struct OwnerTune<double, OpFlux2> {
    static constexpr int B = OPF_FLUX2_BATCH, BC = OPF_FLUX2_CUT_BATCH, WAVES = 0,
                         NT = OPF_FLUX2_THREADS;
    static constexpr bool FOREIGN = true, STREAM = false;
};

// ----------------------------------------------------------- plumbing -- */

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

struct OwnerPtrs {
    const int2 *iblk;       // [ncl] (first edge, count) of the interior block
    const uint32_t *iw;     // interior words by edge (see DevPlan)
    const int *cv_off;      // [ncl+1] cut visits of each cluster
    const int *cv_eid;
    const int *cv_oth;
    const uint16_t *cv_own;
};

template <typename T>
struct Arrays {
    const T *x[kMaxNodeIn];
    double *y[kMaxNodeOut];
    const T *w[kMaxEdgeIn];
    double *wo[3];
};

template <typename T>
Arrays<T> typed(const EdgeArrays &a)
{
    Arrays<T> r;
    for (int k = 0; k < kMaxNodeIn; ++k) r.x[k] = static_cast<const T *>(a.xin[k]);
    for (int k = 0; k < kMaxNodeOut; ++k) r.y[k] = a.yout[k];
    for (int k = 0; k < kMaxEdgeIn; ++k) r.w[k] = static_cast<const T *>(a.w[k]);
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

__device__ __forceinline__ void lds_add(double *p, double v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Element idx of an array at a uniform base, addressed with a 32-bit byte
// offset (idx * sizeof(T) < 2^32), so that no 64-bit address arithmetic runs
// per lane.
template <typename T>
__device__ __forceinline__ T ld(const T *base, int idx)
{
    const uint32_t off = (uint32_t)idx * (uint32_t)sizeof(T);
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + off);
}

template <typename T>
__device__ __forceinline__ void st(T *base, int idx, T v)
{
    const uint32_t off = (uint32_t)idx * (uint32_t)sizeof(T);
    *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + off) = v;
}

// Accesses to data a loop touches once (its edge words and weights, the
// stage's base state and output, a written residual).  With S set they carry
// the non-temporal hint, which keeps them from displacing, in L2, the node
// records that neighbouring workgroups gather.
template <bool S, typename T>
__device__ __forceinline__ T ld1(const T *base, int idx)
{
    if constexpr (S) {
        const uint32_t off = (uint32_t)idx * (uint32_t)sizeof(T);
        return __builtin_nontemporal_load(
            reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + off));
    } else {
        return ld(base, idx);
    }
}

template <bool S, typename T>
__device__ __forceinline__ void st1(T *base, int idx, T v)
{
    if constexpr (S) {
        const uint32_t off = (uint32_t)idx * (uint32_t)sizeof(T);
        __builtin_nontemporal_store(v, reinterpret_cast<T *>(reinterpret_cast<char *>(base) + off));
    } else {
        st(base, idx, v);
    }
}

template <class Op, typename T>
__device__ __forceinline__ void load_stage(const Arrays<T> &a, int g, T gamma, T *s)
{
    T x[Op::NIN];
#pragma unroll
    for (int v = 0; v < Op::NIN; ++v) x[v] = ld(a.x[v], g);
    Op::stage(x, s, gamma);
}

// LDS node records of NS values are kept as planes: W16 planes of 16-byte
// words (plane k holds word k of every record), then at most one plane of
// 8-byte and one of 4-byte words for the rest of the record.  A wavefront
// gathering records of random nodes then spreads each 16-byte read over all 8
// word positions of the 128-byte LDS row, and every read is one ds_read_b128
// (b64, b32 for the tail planes).  Accumulators are NOUT planes of doubles.
template <typename T, int NS>
struct Rec {
    static constexpr int B = NS * (int)sizeof(T);
    static_assert(B % 4 == 0, "records are whole 4-byte words");
    static constexpr int W16 = B / 16, W8 = (B % 16) / 8, W4 = (B % 8) / 4;
};

template <typename T, int NS>
__device__ __forceinline__ void lds_get(const T *base, int rows, int idx, T *out)
{
    using R = Rec<T, NS>;
    alignas(16) unsigned char tmp[R::B];
    const unsigned char *b = reinterpret_cast<const unsigned char *>(base);
#pragma unroll
    for (int k = 0; k < R::W16; ++k) {
        const uint4 w = reinterpret_cast<const uint4 *>(b)[k * rows + idx];
        __builtin_memcpy(tmp + 16 * k, &w, 16);
    }
    b += (size_t)16 * R::W16 * rows;
    if constexpr (R::W8) {
        const uint2 w = reinterpret_cast<const uint2 *>(b)[idx];
        __builtin_memcpy(tmp + 16 * R::W16, &w, 8);
        b += (size_t)8 * rows;
    }
    if constexpr (R::W4) {
        const unsigned w = reinterpret_cast<const unsigned *>(b)[idx];
        __builtin_memcpy(tmp + 16 * R::W16 + 8 * R::W8, &w, 4);
    }
    __builtin_memcpy(out, tmp, R::B);
}

template <typename T, int NS>
__device__ __forceinline__ void lds_put(T *base, int rows, int idx, const T *in)
{
    using R = Rec<T, NS>;
    alignas(16) unsigned char tmp[R::B];
    __builtin_memcpy(tmp, in, R::B);
    unsigned char *b = reinterpret_cast<unsigned char *>(base);
#pragma unroll
    for (int k = 0; k < R::W16; ++k) {
        uint4 w;
        __builtin_memcpy(&w, tmp + 16 * k, 16);
        reinterpret_cast<uint4 *>(b)[k * rows + idx] = w;
    }
    b += (size_t)16 * R::W16 * rows;
    if constexpr (R::W8) {
        uint2 w;
        __builtin_memcpy(&w, tmp + 16 * R::W16, 8);
        reinterpret_cast<uint2 *>(b)[idx] = w;
        b += (size_t)8 * rows;
    }
    if constexpr (R::W4) {
        unsigned w;
        __builtin_memcpy(&w, tmp + 16 * R::W16 + 8 * R::W8, 4);
        reinterpret_cast<unsigned *>(b)[idx] = w;
    }
}

// LDS bytes of `rows` records, rounded up to 16 (the accumulators follow).
template <typename T, class Op>
__host__ __device__ constexpr size_t stage_bytes(int rows)
{
    return ((size_t)Rec<T, Op::NS>::B * rows + 15) / 16 * 16;
}

template <typename T, class Op>
constexpr size_t lds_bytes(int rows)
{
    return stage_bytes<T, Op>(rows) + (size_t)Op::NOUT * rows * sizeof(double);
}

// ---------------------------------------------------- coloured kernel -- */

template <typename T, class Op, int NT, int EPT, bool LDSAT>
__global__ __launch_bounds__(NT) void k_edge_coloured(PlanPtrs p, Arrays<T> a, T gamma, int cbase,
                                                      int ncb, int remap)
{
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NY = Op::MODE == GEN ? 2 * Op::NOUT : Op::NOUT;
    const int umax = p.umax;
    T *ss = reinterpret_cast<T *>(smem);
    double *sy = reinterpret_cast<double *>(smem + stage_bytes<T, Op>(umax));

    const int k = remap ? xcd_map((int)blockIdx.x, ncb) : (int)blockIdx.x;
    const int b = p.colour_blocks[cbase + k];
    const int e0 = p.block_off[b], ne = p.block_off[b + 1] - e0;
    const int u0 = p.uniq_off[b], nu = p.uniq_off[b + 1] - u0;

    // stage the partition's nodes, clear its accumulator
    for (int u = threadIdx.x; u < nu; u += NT) {
        T s[Op::NS];
        load_stage<Op>(a, p.uniq[u0 + u], gamma, s);
        lds_put<T, Op::NS>(ss, umax, u, s);
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
            T si[Op::NS], sj[Op::NS], n[Op::NW];
            lds_get<T, Op::NS>(ss, umax, li[t], si);
            lds_get<T, Op::NS>(ss, umax, lj[t], sj);
#pragma unroll
            for (int d = 0; d < Op::NW; ++d) n[d] = ld(a.w[d], e0 + e);
            double wo[3] = {0.0, 0.0, 0.0};
            Op::edge(si, sj, n, gamma, y[t], y[t] + (NY - Op::NOUT), wo);
            if (Op::NWOUT) {
#pragma unroll
                for (int d = 0; d < 3; ++d) a.wo[d][e0 + e] = wo[d];
            }
            if (LDSAT) {
#pragma unroll
                for (int v = 0; v < Op::NOUT; ++v) {
                    const double yi = y[t][v];
                    const double yj = Op::MODE == ANTI ? -yi : Op::MODE == SAME ? yi : y[t][Op::NOUT + v];
                    lds_add(&sy[v * umax + li[t]], yi);
                    lds_add(&sy[v * umax + lj[t]], yj);
                }
            }
        }
    }
    if (LDSAT) {
        __syncthreads();
    } else {
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
    }

    // add the partition's accumulator to HBM (no other partition of this
    // colour touches these nodes)
    for (int u = threadIdx.x; u < nu; u += NT) {
        const int g = p.uniq[u0 + u];
#pragma unroll
        for (int v = 0; v < Op::NOUT; ++v) a.y[v][g] += sy[v * umax + u];
    }
}

// ------------------------------------------------------ atomic kernel -- */

template <typename T, class Op>
__global__ __launch_bounds__(256) void k_edge_atomic(const int2 *__restrict__ e2n, int E,
                                                     Arrays<T> a, T gamma, int remap)
{
    const int blk = remap ? xcd_map((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x;
    const int e = blk * 256 + (int)threadIdx.x;
    if (e >= E) return;
    const int2 ij = e2n[e];
    T si[Op::NS], sj[Op::NS], n[Op::NW];
    load_stage<Op>(a, ij.x, gamma, si);
    load_stage<Op>(a, ij.y, gamma, sj);
#pragma unroll
    for (int d = 0; d < Op::NW; ++d) n[d] = ld(a.w[d], e);
    constexpr int NY = Op::MODE == GEN ? 2 * Op::NOUT : Op::NOUT;
    double y[NY];
    double wo[3] = {0.0, 0.0, 0.0};
    Op::edge(si, sj, n, gamma, y, y + (NY - Op::NOUT), wo);
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

// ------------------------------------------------------- flat kernel -- */

// One colour of the flat colouring: one thread per edge, both ends gathered
// from HBM, both increments added with a plain read-add-write (no other edge
// of this colour touches either end).
template <typename T, class Op>
__global__ __launch_bounds__(256) void k_edge_flat(const int2 *__restrict__ e2n,
                                                   const int *__restrict__ eids, int n, Arrays<T> a,
                                                   T gamma)
{
    const int t = (int)blockIdx.x * 256 + (int)threadIdx.x;
    if (t >= n) return;
    const int e = eids[t];
    const int2 ij = ld(e2n, e);
    T si[Op::NS], sj[Op::NS], w[Op::NW];
    load_stage<Op>(a, ij.x, gamma, si);
    load_stage<Op>(a, ij.y, gamma, sj);
#pragma unroll
    for (int d = 0; d < Op::NW; ++d) w[d] = ld(a.w[d], e);
    constexpr int NY = Op::MODE == GEN ? 2 * Op::NOUT : Op::NOUT;
    double y[NY];
    double wo[3] = {0.0, 0.0, 0.0};
    Op::edge(si, sj, w, gamma, y, y + (NY - Op::NOUT), wo);
#pragma unroll
    for (int v = 0; v < Op::NOUT; ++v) {
        const double yi = y[v];
        const double yj = Op::MODE == ANTI ? -yi : Op::MODE == SAME ? yi : y[Op::NOUT + v];
        st(a.y[v], ij.x, ld(a.y[v], ij.x) + yi);
        st(a.y[v], ij.y, ld(a.y[v], ij.y) + yj);
    }
    if (Op::NWOUT) {
#pragma unroll
        for (int d = 0; d < 3; ++d) st(a.wo[d], e, wo[d]);
    }
}

// Sum over a workgroup of NWAVE wavefronts; out[v] in a fixed order.
template <int NV, int NWAVE = 4>
__device__ __forceinline__ void block_sum(double (&acc)[NV], double *out)
{
    __shared__ double red[NWAVE][NV];
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
        double t = red[0][v];
#pragma unroll
        for (int w = 1; w < NWAVE; ++w) t += red[w][v];
        out[v] = t;
    }
}

// out[0..5] = the sums over the workgroup's NT threads of acc[0..5], through
// LDS (buf: 6 * NT doubles, free for this use) in a fixed tree: 64 lanes x 8,
// then 8, then the last 8.  Three LDS rounds instead of the 36 dependent
// cross-lane shuffles of a wavefront reduction of six doubles.
template <int NT>
__device__ __forceinline__ void lds_sum6(const double (&acc)[6], double *buf, double *out)
{
    static_assert(NT == 512, "the tree is laid out for 512 threads");
    const int t = threadIdx.x;
    __syncthreads();  // buf may still be read
#pragma unroll
    for (int k = 0; k < 6; ++k) buf[k * NT + t] = acc[k];
    __syncthreads();
    if (t < 6 * 64) {
        const int k = t >> 6, j = t & 63;
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < NT / 64; ++i) s += buf[k * NT + j + 64 * i];
        buf[k * NT + j] = s;
    }
    __syncthreads();
    if (t < 6 * 8) {
        const int k = t >> 3, j = t & 7;
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < 8; ++i) s += buf[k * NT + j + 8 * i];
        buf[k * NT + j] = s;
    }
    __syncthreads();
    if (t < 6) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < 8; ++i) s += buf[t * NT + i];
        out[t] = s;
    }
}

// ------------------------------------------------------- owner kernel -- */

// One workgroup per cluster of K consecutive nodes runs every edge with an
// end in the cluster and adds only into its own nodes' LDS accumulators, then
// writes each node's total once.  Two loops, each uniform across a wavefront:
//   (1) the interior block: edges with both ends in the cluster, read through
//       4-byte words of local offsets; both records come from LDS and both
//       ends are updated (the word's flag picks which first: bank spreading);
//   (2) the cut visits: one (edge, owned end) pair each; the owned end's
//       record comes from LDS, the other end's state is gathered from memory
//       and staged in registers.  The flux is evaluated with the owned end as
//       the first node: F(a, b, w) = -F(b, a, -w) for every kernel here (the
//       edge inputs flip sign with the orientation), so a visit whose owned
//       end is the edge's second node negates its edge inputs and adds the
//       first-node result.  An edge joining two clusters runs in both.
// KC > 0 fixes the cluster size at compile time (LDS addresses become
// immediate offsets); KC = 0 takes it from the launch.
__host__ __device__ constexpr int owner_acc_rows(int K) { return K; }

// The stage update fused into the owner loop: each workgroup turns its nodes'
// totals straight into q = q0 - adt * res / vol (adt * dt_i with per-node
// steps) and a partial sum of res^2 per component, so the residual never
// goes to HBM.
template <typename T>
struct StagePtrs {
    const T *q0[6];
    T *q[6];
    const double *vol;
    const double *dt;  // per-node steps or null
    double adt;
    double *partial;   // [ncl][6]
};

// HALVES: two workgroups per cluster, b and b + 8 of each 16 (dispatched to the
// same XCD, so that the second reads the cluster's edges from L2), each
// running Op on its half of the node inputs and outputs (grid: 16 per 8
// clusters, rounded up; the surplus exits).  HINT: the non-temporal hints
// (where the op takes them).
template <typename T, class Op, int NT, int KC, bool STAGE = false, bool HALVES = false,
          bool HINT = false>
__global__ __launch_bounds__(NT, (OwnerTune<T, Op>::WAVES > 0 ? OwnerTune<T, Op>::WAVES : 1)) void k_edge_owner(
    OwnerPtrs p, Arrays<T> a0, T gamma, int N, int Kr, int ncl, int remap, int overwrite,
    StagePtrs<T> sp = {})
{
    constexpr int B = OwnerTune<T, Op>::B;
    constexpr bool S = HINT && OwnerTune<T, Op>::STREAM;
    const int K = KC > 0 ? KC : Kr;
    extern __shared__ __align__(16) unsigned char smem[];
    T *ss = reinterpret_cast<T *>(smem);
    double *sy = reinterpret_cast<double *>(smem + stage_bytes<T, Op>(K));

    int c;
    Arrays<T> a = a0;
    if constexpr (HALVES) {
        const int b = (int)blockIdx.x, k = (b & 7) + 8 * (b >> 4), h = (b >> 3) & 1;
        if (k >= ncl) return;
        c = remap ? xcd_map(k, ncl) : k;
        if (h) {
#pragma unroll
            for (int v = 0; v < Op::NIN; ++v) a.x[v] = a0.x[Op::NIN + v];
#pragma unroll
            for (int v = 0; v < Op::NOUT; ++v) a.y[v] = a0.y[Op::NOUT + v];
        }
    } else {
        c = remap ? xcd_map((int)blockIdx.x, ncl) : (int)blockIdx.x;
    }
    const int v0 = c * K, nown = min(K, N - v0);
    // stage the owned nodes (contiguous ids: coalesced), clear the accumulator
    for (int v = threadIdx.x; v < nown; v += NT) {
        T rec[Op::NS];
        load_stage<Op>(a, v0 + v, gamma, rec);
        lds_put<T, Op::NS>(ss, K, v, rec);
#pragma unroll
        for (int k = 0; k < Op::NOUT; ++k) sy[k * K + v] = 0.0;
    }
    __syncthreads();

    // (1) interior block
    const int2 ib = p.iblk[c];
    for (int k0 = threadIdx.x; k0 < ib.y; k0 += NT * B) {
        uint32_t wd[B];
        T w[B][Op::NW];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int k = k0 + b * NT;
            if (k < ib.y) {
                wd[b] = ld1<S>(p.iw, ib.x + k);
#pragma unroll
                for (int d = 0; d < Op::NW; ++d) w[b][d] = ld1<S>(a.w[d], ib.x + k);
            }
        }
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int k = k0 + b * NT;
            if (k >= ib.y) continue;
            const int li = (int)(wd[b] & 0x1fffu), lj = (int)((wd[b] >> 16) & 0x1fffu);
            const uint32_t swp = wd[b] >> 31;
            T si[Op::NS], sj[Op::NS];
            lds_get<T, Op::NS>(ss, K, li, si);
            lds_get<T, Op::NS>(ss, K, lj, sj);
            double y[Op::NOUT], yj[Op::NOUT];
            double wo[3] = {0.0, 0.0, 0.0};
            Op::edge(si, sj, w[b], gamma, y, yj, wo);
            const int la = swp ? lj : li, lb = swp ? li : lj;
#pragma unroll
            for (int v = 0; v < Op::NOUT; ++v) {
                if constexpr (Op::MODE == ANTI) {
                    const double ya = flip(y[v], swp);
                    lds_add(&sy[v * K + la], ya);
                    lds_add(&sy[v * K + lb], -ya);
                } else if constexpr (Op::MODE == SAME) {
                    lds_add(&sy[v * K + la], y[v]);
                    lds_add(&sy[v * K + lb], y[v]);
                } else {
                    lds_add(&sy[v * K + la], swp ? yj[v] : y[v]);
                    lds_add(&sy[v * K + lb], swp ? y[v] : yj[v]);
                }
            }
            if constexpr (Op::NWOUT > 0) {
#pragma unroll
                for (int d = 0; d < 3; ++d) st1<S>(a.wo[d], ib.x + k, wo[d]);
            }
        }
    }

    // (2) cut visits
    constexpr int BC = OwnerTune<T, Op>::BC;
    const int s0 = p.cv_off[c], ns = p.cv_off[c + 1] - s0;
    for (int k0 = threadIdx.x; k0 < ns; k0 += NT * BC) {
        int eid[BC], oth[BC], own[BC];
#pragma unroll
        for (int b = 0; b < BC; ++b) {
            const int k = k0 + b * NT;
            eid[b] = -1;
            if (k < ns) {
                eid[b] = ld1<S>(p.cv_eid, s0 + k);
                oth[b] = ld1<S>(p.cv_oth, s0 + k);
                own[b] = (int)ld1<S>(p.cv_own, s0 + k);
            }
        }
        T w[BC][Op::NW], xf[BC][Op::NIN];
#pragma unroll
        for (int b = 0; b < BC; ++b) {
            if (eid[b] < 0) continue;
            const int g = oth[b] & 0x7fffffff;
#pragma unroll
            for (int d = 0; d < Op::NW; ++d) w[b][d] = ld(a.w[d], eid[b]);
#pragma unroll
            for (int v = 0; v < Op::NIN; ++v) xf[b][v] = ld(a.x[v], g);
        }
#pragma unroll
        for (int b = 0; b < BC; ++b) {
            if (eid[b] < 0) continue;
            const uint32_t second = (uint32_t)oth[b] >> 31;
            T so[Op::NS], sf[Op::NS], wf[Op::NW];
            lds_get<T, Op::NS>(ss, K, own[b], so);
            Op::stage(xf[b], sf, gamma);
#pragma unroll
            for (int d = 0; d < Op::NW; ++d) wf[d] = flip(w[b][d], second);
            double y[Op::NOUT], yj[Op::NOUT];
            double wo[3] = {0.0, 0.0, 0.0};
            Op::edge(so, sf, wf, gamma, y, yj, wo);
#pragma unroll
            for (int v = 0; v < Op::NOUT; ++v) lds_add(&sy[v * K + own[b]], y[v]);
            // a direct output is written by the visit from the smaller end only
            if constexpr (Op::NWOUT > 0) {
                if (v0 + own[b] < (oth[b] & 0x7fffffff)) {
#pragma unroll
                    for (int d = 0; d < 3; ++d) st1<S>(a.wo[d], eid[b], flip(wo[d], second));
                }
            }
        }
    }
    // fused stage: issue this thread's node's q0 and vol loads before the
    // barrier, so that they arrive while the slower lanes finish their edges
    // (one node per thread when K <= NT; held in registers only from here on)
    [[maybe_unused]] double pq0[6], pvol = 1.0;
    if constexpr (STAGE) {
        if (K <= NT && (int)threadIdx.x < nown) {
#pragma unroll
            for (int k = 0; k < 6; ++k) pq0[k] = (double)ld1<S>(sp.q0[k], v0 + (int)threadIdx.x);
            pvol = ld1<S>(sp.vol, v0 + (int)threadIdx.x);
        }
    }
    __syncthreads();
    if constexpr (STAGE) {
        double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (int v = threadIdx.x; v < nown; v += NT) {
            const int g = v0 + v;
            const bool pre = K <= NT;
            const double vi = pre ? pvol : ld1<S>(sp.vol, g);
            const double adt = sp.dt ? sp.adt * ld(sp.dt, g) : sp.adt;
            const double step = adt / vi;  // one division per node
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                const double r = sy[k * K + v];
                acc[k] += r * r;
                const double base = pre ? pq0[k] : (double)ld1<S>(sp.q0[k], g);
                st1<S>(sp.q[k], g, (T)(base - step * r));
            }
        }
        bool done = false;
        if constexpr (NT == 512) {
            if (K >= NT) {  // the accumulators hold 6 * NT doubles
                lds_sum6<NT>(acc, sy, sp.partial + 6 * c);
                done = true;
            }
        }
        if (!done) block_sum<6, NT / 64>(acc, sp.partial + 6 * c);
    } else {
        for (int v = threadIdx.x; v < nown; v += NT) {
#pragma unroll
            for (int k = 0; k < Op::NOUT; ++k) {
                const double acc = sy[k * K + v];
                st1<S>(a.y[k], v0 + v, overwrite ? acc : ld(a.y[k], v0 + v) + acc);
            }
        }
    }
}

// ------------------------------------------------------ reductions -- */

template <typename T>
struct RkPtrs {
    const T *q0[6];
    double *res[6];
    const double *vol;
    T *q[6];
    const double *dt;  // per-node steps (local time stepping) or null
};

template <typename T>
__global__ __launch_bounds__(kRkThreads) void k_rk_stage(int N, RkPtrs<T> a, double alpha_dt,
                                                         double *partial, int keep_res)
{
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const int stride = (int)gridDim.x * kRkThreads;
    for (int i = (int)blockIdx.x * kRkThreads + (int)threadIdx.x; i < N; i += stride) {
        const double vi = a.vol[i];
        const double adt = a.dt ? alpha_dt * a.dt[i] : alpha_dt;
        const double step = adt / vi;  // one division per node
#pragma unroll
        for (int v = 0; v < 6; ++v) {
            const double r = a.res[v][i];
            acc[v] += r * r;
            a.q[v][i] = (T)((double)a.q0[v][i] - step * r);
            if (!keep_res) a.res[v][i] = 0.0;
        }
    }
    block_sum<6>(acc, partial + 6 * blockIdx.x);
}

__global__ __launch_bounds__(kRkThreads) void k_local_dt(int N, const double *__restrict__ vol,
                                                         const double *__restrict__ lam, double cfl,
                                                         double *__restrict__ dt)
{
    const int stride = (int)gridDim.x * kRkThreads;
    for (int i = (int)blockIdx.x * kRkThreads + (int)threadIdx.x; i < N; i += stride)
        dt[i] = cfl * vol[i] / lam[i];
}

// ss[0..5] += the sum of nparts rows of 6 partial sums (rows at buf +
// kSumTail).  Workgroup g of kSumGroups sums the rows [g R, (g+1) R), each
// thread a fixed stride of them, then through a fixed LDS tree, into
// buf[6 g ..]; the last workgroup to finish adds the kSumGroups sums in
// order.  Every order is fixed, so the result is the same on every run.
constexpr int kSumThreads = 256;

__global__ __launch_bounds__(kSumThreads) void k_sum_partials(int nparts, double *buf, double *ss)
{
    const double *rows = buf + kSumTail;
    unsigned int *counter = reinterpret_cast<unsigned int *>(buf + 6 * kSumGroups);
    const int g = (int)blockIdx.x, t = (int)threadIdx.x;
    const int per = (nparts + kSumGroups - 1) / kSumGroups;
    const int r0 = g * per, r1 = min(nparts, r0 + per);
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    constexpr int U = 4;  // rows whose loads are in flight together
    for (int r = r0 + t; r < r1; r += kSumThreads * U) {
        double2 v[U][3];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = r + u * kSumThreads;
            const double2 *p2 = reinterpret_cast<const double2 *>(rows + 6 * (size_t)k);
#pragma unroll
            for (int w = 0; w < 3; ++w) v[u][w] = k < r1 ? p2[w] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int w = 0; w < 3; ++w) {
                acc[2 * w] += v[u][w].x;
                acc[2 * w + 1] += v[u][w].y;
            }
    }
    // fixed tree through LDS: 64 lanes x 4 per component (384 sums over 256
    // threads), then 8 x 8, then 8
    __shared__ double red[6 * kSumThreads];
    __shared__ int last;
#pragma unroll
    for (int v = 0; v < 6; ++v) red[v * kSumThreads + t] = acc[v];
    __syncthreads();
    for (int idx = t; idx < 6 * 64; idx += kSumThreads) {
        const int v = idx >> 6, j = idx & 63;
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < kSumThreads / 64; ++i) s += red[v * kSumThreads + j + 64 * i];
        red[v * kSumThreads + j] = s;
    }
    __syncthreads();
    if (t < 6 * 8) {
        const int v = t >> 3, j = t & 7;
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < 8; ++i) s += red[v * kSumThreads + j + 8 * i];
        red[v * kSumThreads + j] = s;
    }
    __syncthreads();
    if (t < 6) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < 8; ++i) s += red[t * kSumThreads + i];
        buf[6 * g + t] = s;
    }
    // publish this group's sums, then count it; the last group sees all
    __threadfence();
    __syncthreads();
    if (t == 0) last = atomicAdd(counter, 1u) == (unsigned int)(kSumGroups - 1);
    __syncthreads();
    if (!last) return;
    __threadfence();
    if (t < 6) {
        const volatile double *vb = buf;
        double s = 0.0;
        for (int i = 0; i < kSumGroups; ++i) s += vb[6 * i + t];
        ss[t] += s;
    }
    if (t == 0) *counter = 0u;
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

template <typename T, class Op, int NT, int EPT, bool LDSAT>
int run_coloured(const DevPlan &P, const EdgeArrays &a, double gamma, hipStream_t st,
                 const LaunchOpts &lo)
{
    const size_t lds = lds_bytes<T, Op>(P.umax);
    const Arrays<T> ta = typed<T>(a);
    const PlanPtrs pp = plan_ptrs(P);
    for (int c = 0; c < P.nc; ++c) {
        const int n = P.colour_off[c + 1] - P.colour_off[c];
        if (n <= 0) continue;
        hipLaunchKernelGGL((k_edge_coloured<T, Op, NT, EPT, LDSAT>), dim3(n), dim3(NT), lds, st,
                           pp, ta, (T)gamma, P.colour_off[c], n, lo.xcd_remap);
    }
    return (int)hipGetLastError();
}

template <typename T, class Op, bool LDSAT>
int run_coloured_bs(const DevPlan &P, const EdgeArrays &a, double gamma, hipStream_t st,
                    const LaunchOpts &lo)
{
    switch (P.block_size) {
    case 64: return run_coloured<T, Op, 64, 1, LDSAT>(P, a, gamma, st, lo);
    case 128: return run_coloured<T, Op, 128, 1, LDSAT>(P, a, gamma, st, lo);
    case 256: return run_coloured<T, Op, 256, 1, LDSAT>(P, a, gamma, st, lo);
    case 512: return run_coloured<T, Op, 256, 2, LDSAT>(P, a, gamma, st, lo);
    case 1024: return run_coloured<T, Op, 256, 4, LDSAT>(P, a, gamma, st, lo);
    case 2048: return run_coloured<T, Op, 256, 8, LDSAT>(P, a, gamma, st, lo);
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
int run_flat(const DevPlan &P, const EdgeArrays &a, double gamma, hipStream_t st)
{
    if (P.nflat <= 0) return (int)hipErrorInvalidValue;
    for (int c = 0; c < P.nflat; ++c) {
        const int64_t off = P.flat_off[c], n = P.flat_off[c + 1] - off;
        if (n <= 0) continue;
        hipLaunchKernelGGL((k_edge_flat<T, Op>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                           P.e2n, P.flat_eid + off, (int)n, typed<T>(a), (T)gamma);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return (int)e;
    }
    return 0;
}

template <typename T, class Op>
constexpr size_t owner_dyn_lds(int K)
{
    return stage_bytes<T, Op>(K) + (size_t)Op::NOUT * owner_acc_rows(K) * sizeof(double);
}

OwnerPtrs owner_ptrs(const DevPlan &P, bool foreign)
{
    if (foreign) return OwnerPtrs{P.iblk, P.iw, P.cv_off, P.cvf_eid, P.cvf_oth, P.cvf_own};
    return OwnerPtrs{P.iblk, P.iw, P.cv_off, P.cv_eid, P.cv_oth, P.cv_own};
}

// Cluster size fixed at compile time for the default plan.
constexpr int kOwnerKC = 512;

// The device's last-level cache (MALL, 256 MB).  A loop whose arrays fit in
// it finds them there again at its next launch, which the non-temporal hints
// would spoil (the FP32 flux loops of a 1M-node mesh: 12-20 % slower with
// them); a larger loop streams through it, and the hints keep its L2 for the
// halo records.
constexpr double kMallBytes = 256.0 * 1024 * 1024;

// Whether the owner loop of Op over plan P takes the non-temporal hints: its
// bytes per launch (edge map and inputs; node inputs and outputs, or for the
// fused stage q, q0, the new state and vol) exceed the last-level cache.
template <typename T, class Op>
bool owner_streams(const DevPlan &P, bool stage)
{
    if (!OwnerTune<T, Op>::STREAM) return false;
    const double per_node = stage ? 3.0 * 6 * sizeof(T) + sizeof(double)
                                  : (double)Op::NIN * sizeof(T) + Op::NOUT * sizeof(double);
    const double bytes = (double)P.E * (8.0 + Op::NW * sizeof(T)) + (double)P.N * per_node;
    return bytes > kMallBytes;
}

// Launches the owner kernel of op O (KC: compile-time cluster size or 0).
template <typename T, class O, int NT, int KC, bool STAGE, bool H>
void launch_owner_kc(bool hint, int grid, size_t lds, hipStream_t st, const OwnerPtrs &op,
                     const Arrays<T> &a, T gamma, const DevPlan &P, const LaunchOpts &lo,
                     int overwrite, const StagePtrs<T> &sp)
{
    if constexpr (OwnerTune<T, O>::STREAM) {
        if (hint) {
            hipLaunchKernelGGL((k_edge_owner<T, O, NT, KC, STAGE, H, true>), dim3(grid), dim3(NT),
                               lds, st, op, a, gamma, P.N, P.K, P.ncl, lo.xcd_remap, overwrite, sp);
            return;
        }
    }
    hipLaunchKernelGGL((k_edge_owner<T, O, NT, KC, STAGE, H, false>), dim3(grid), dim3(NT), lds,
                       st, op, a, gamma, P.N, P.K, P.ncl, lo.xcd_remap, overwrite, sp);
}

template <typename T, class O, int NT, bool STAGE, bool H>
void launch_owner(bool hint, int grid, size_t lds, hipStream_t st, const OwnerPtrs &op,
                  const Arrays<T> &a, T gamma, const DevPlan &P, const LaunchOpts &lo,
                  int overwrite, const StagePtrs<T> &sp)
{
    if (P.K == kOwnerKC)
        launch_owner_kc<T, O, NT, kOwnerKC, STAGE, H>(hint, grid, lds, st, op, a, gamma, P, lo,
                                                      overwrite, sp);
    else
        launch_owner_kc<T, O, NT, 0, STAGE, H>(hint, grid, lds, st, op, a, gamma, P, lo, overwrite,
                                               sp);
}

template <typename T, class Op>
int run_owner(const DevPlan &P, const EdgeArrays &a, double gamma, hipStream_t st,
              const LaunchOpts &lo)
{
    if (!P.owner_ok || P.ncl <= 0) return (int)hipErrorInvalidValue;
    using O = typename OwnerOp<Op>::type;
    constexpr bool H = OwnerOp<Op>::HALVES;
    const size_t lds = owner_dyn_lds<T, O>(P.K);
    const OwnerPtrs op = owner_ptrs(P, OwnerTune<T, O>::FOREIGN);
    constexpr int NT = OwnerTune<T, O>::NT;
    const int grid = H ? 16 * ((P.ncl + 7) / 8) : P.ncl;
    launch_owner<T, O, NT, false, H>(owner_streams<T, O>(P, false), grid, lds, st, op, typed<T>(a),
                                     (T)gamma, P, lo, lo.overwrite, StagePtrs<T>{});
    return (int)hipGetLastError();
}

template <typename T>
int run_owner_stage(const DevPlan &P, const EdgeArrays &a, const NodeArrays &na, double gamma,
                    double adt, double *ss, double *partial, hipStream_t st, const LaunchOpts &lo)
{
    if (!P.owner_ok || P.ncl <= 0 || !partial) return (int)hipErrorInvalidValue;
    const size_t lds = owner_dyn_lds<T, OpFlux>(P.K);
    const OwnerPtrs op = owner_ptrs(P, OwnerTune<T, OpFlux>::FOREIGN);
    StagePtrs<T> sp;
    for (int k = 0; k < 6; ++k) {
        sp.q0[k] = static_cast<const T *>(na.q0[k]);
        sp.q[k] = static_cast<T *>(na.q[k]);
    }
    sp.vol = na.vol;
    sp.dt = na.dt;
    sp.adt = adt;
    sp.partial = partial + kSumTail;
    launch_owner<T, OpFlux, kOwnerThreads, true, false>(owner_streams<T, OpFlux>(P, true), P.ncl,
                                                        lds, st, op, typed<T>(a), (T)gamma, P, lo,
                                                        0, sp);
    hipLaunchKernelGGL(k_sum_partials, dim3(kSumGroups), dim3(kSumThreads), 0, st, P.ncl, partial,
                       ss);
    return (int)hipGetLastError();
}

template <typename T, class Op>
int run_edge(int variant, const DevPlan &P, const EdgeArrays &a, double gamma, hipStream_t st,
             const LaunchOpts &lo)
{
    switch (variant) {
    case V_COLOURED: return run_coloured_bs<T, Op, false>(P, a, gamma, st, lo);
    case V_COLOURED_LDS_ATOMIC: return run_coloured_bs<T, Op, true>(P, a, gamma, st, lo);
    case V_ATOMIC: return run_atomic<T, Op>(P, a, gamma, st, lo);
    case V_OWNER: return run_owner<T, Op>(P, a, gamma, st, lo);
    case V_FLAT: return run_flat<T, Op>(P, a, gamma, st);
    default: return (int)hipErrorInvalidValue;
    }
}

// Lets kernel f use up to `total` bytes of LDS, static part included.
int raise_one(const void *f, size_t total)
{
    hipFuncAttributes attr;
    hipError_t e = hipFuncGetAttributes(&attr, f);
    if (e != hipSuccess) return (int)e;
    if (attr.sharedSizeBytes >= total) return 0;
    e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(total - attr.sharedSizeBytes));
    return (int)e;
}

template <typename T, class Op, bool LDSAT>
int raise_coloured(size_t bytes)
{
    const void *fns[] = {
        reinterpret_cast<const void *>(&k_edge_coloured<T, Op, 64, 1, LDSAT>),
        reinterpret_cast<const void *>(&k_edge_coloured<T, Op, 128, 1, LDSAT>),
        reinterpret_cast<const void *>(&k_edge_coloured<T, Op, 256, 1, LDSAT>),
        reinterpret_cast<const void *>(&k_edge_coloured<T, Op, 256, 2, LDSAT>),
        reinterpret_cast<const void *>(&k_edge_coloured<T, Op, 256, 4, LDSAT>),
        reinterpret_cast<const void *>(&k_edge_coloured<T, Op, 256, 8, LDSAT>)};
    for (const void *f : fns) {
        int e = raise_one(f, bytes);
        if (e) return e;
    }
    return 0;
}

template <typename T, class O, int NT, bool STAGE, bool H>
int raise_owner(size_t bytes)
{
    int rc = raise_one(reinterpret_cast<const void *>(&k_edge_owner<T, O, NT, 0, STAGE, H, false>), bytes);
    if (!rc)
        rc = raise_one(reinterpret_cast<const void *>(&k_edge_owner<T, O, NT, kOwnerKC, STAGE, H, false>),
                       bytes);
    if constexpr (OwnerTune<T, O>::STREAM) {
        if (!rc)
            rc = raise_one(reinterpret_cast<const void *>(&k_edge_owner<T, O, NT, 0, STAGE, H, true>),
                           bytes);
        if (!rc)
            rc = raise_one(
                reinterpret_cast<const void *>(&k_edge_owner<T, O, NT, kOwnerKC, STAGE, H, true>), bytes);
    }
    return rc;
}

template <typename T, class Op>
int raise_all(size_t bytes)
{
    int rc = raise_coloured<T, Op, false>(bytes);
    if (!rc) rc = raise_coloured<T, Op, true>(bytes);
    using O = typename OwnerOp<Op>::type;
    constexpr bool H = OwnerOp<Op>::HALVES;
    constexpr int NT = OwnerTune<T, O>::NT;
    if (!rc) rc = raise_owner<T, O, NT, false, H>(bytes);
    if constexpr (std::is_same<Op, OpFlux>::value) {
        if (!rc) rc = raise_owner<T, Op, kOwnerThreads, true, false>(bytes);
    }
    return rc;
}

size_t owner_dyn_lds_bytes(int op, bool fp32, int K)
{
    if (op == OP_ADJOINT) return owner_dyn_lds<double, OpAdjoint>(K);
    if (op == OP_GRAD) return owner_dyn_lds<double, OpGradH>(K);
    if (op == OP_FLUX2) return owner_dyn_lds<double, OpFlux2>(K);
    if (op == OP_SPECRAD) return fp32 ? owner_dyn_lds<float, OpSpecrad>(K) : owner_dyn_lds<double, OpSpecrad>(K);
    return fp32 ? owner_dyn_lds<float, OpFlux>(K) : owner_dyn_lds<double, OpFlux>(K);
}

// LDS of an owner workgroup: the dynamic part plus a static allowance for the
// fused stage's reduction.
size_t owner_lds_bytes(int op, bool fp32, int K)
{
    return owner_dyn_lds_bytes(op, fp32, K) + 2048;
}

}  // namespace

size_t edge_lds_bytes(int op, bool fp32, int variant, int umax, int K)
{
    if (variant == V_ATOMIC || variant == V_FLAT) return 0;
    if (variant == V_OWNER) return owner_lds_bytes(op, fp32, K);
    const int rows = umax;
    if (op == OP_ADJOINT) return lds_bytes<double, OpAdjoint>(rows);
    if (op == OP_GRAD) return lds_bytes<double, OpGrad>(rows);
    if (op == OP_FLUX2) return lds_bytes<double, OpFlux2>(rows);
    if (op == OP_SPECRAD)
        return fp32 ? lds_bytes<float, OpSpecrad>(rows) : lds_bytes<double, OpSpecrad>(rows);
    return fp32 ? lds_bytes<float, OpFlux>(rows) : lds_bytes<double, OpFlux>(rows);
}

int set_lds_limit(size_t bytes)
{
    int rc = raise_all<double, OpFlux>(bytes);
    if (!rc) rc = raise_all<float, OpFlux>(bytes);
    if (!rc) rc = raise_all<double, OpSpecrad>(bytes);
    if (!rc) rc = raise_all<float, OpSpecrad>(bytes);
    if (!rc) rc = raise_all<double, OpAdjoint>(bytes);
    if (!rc) rc = raise_all<double, OpGrad>(bytes);
    if (!rc) rc = raise_all<double, OpFlux2>(bytes);
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
    case OP_GRAD:
        if (fp32) return (int)hipErrorInvalidValue;
        return run_edge<double, OpGrad>(variant, P, a, gamma, st, lo);
    case OP_FLUX2:
        if (fp32) return (int)hipErrorInvalidValue;
        return run_edge<double, OpFlux2>(variant, P, a, gamma, st, lo);
    default: return (int)hipErrorInvalidValue;
    }
}

int launch_edge_stage(bool fp32, const DevPlan &P, const EdgeArrays &a, const NodeArrays &na,
                      double gamma, double adt, double *ss, double *partial, hipStream_t st,
                      const LaunchOpts &lo)
{
    return fp32 ? run_owner_stage<float>(P, a, na, gamma, adt, ss, partial, st, lo)
                : run_owner_stage<double>(P, a, na, gamma, adt, ss, partial, st, lo);
}

int static_scratch_address(double **out)
{
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return (int)e;
    *out = static_cast<double *>(p);
    return 0;
}

template <typename T>
static int run_rk(int N, const NodeArrays &a, double alpha_dt, double *ss, double *partial,
                  bool keep_res, hipStream_t st)
{
    RkPtrs<T> p;
    for (int v = 0; v < 6; ++v) {
        p.q0[v] = static_cast<const T *>(a.q0[v]);
        p.res[v] = a.res[v];
        p.q[v] = static_cast<T *>(a.q[v]);
    }
    p.vol = a.vol;
    p.dt = a.dt;
    const int grid = std::min(kRkBlocks, std::max(1, (N + kRkThreads - 1) / kRkThreads));
    hipLaunchKernelGGL((k_rk_stage<T>), dim3(grid), dim3(kRkThreads), 0, st, N, p, alpha_dt,
                       partial + kSumTail, keep_res ? 1 : 0);
    hipLaunchKernelGGL(k_sum_partials, dim3(kSumGroups), dim3(kSumThreads), 0, st, grid, partial,
                       ss);
    return (int)hipGetLastError();
}

int launch_rk_stage(bool fp32, int N, const NodeArrays &a, double alpha_dt, double *ss,
                    double *partial, bool keep_res, hipStream_t st)
{
    return fp32 ? run_rk<float>(N, a, alpha_dt, ss, partial, keep_res, st)
                : run_rk<double>(N, a, alpha_dt, ss, partial, keep_res, st);
}

int launch_dt_min(int N, const double *vol, const double *lam, double cfl, double *dt,
                  double *partial, hipStream_t st)
{
    const int grid = std::min(kRkBlocks, std::max(1, (N + kRkThreads - 1) / kRkThreads));
    hipLaunchKernelGGL(k_dt_min, dim3(grid), dim3(kRkThreads), 0, st, N, vol, lam,
                       partial + kSumTail);
    hipLaunchKernelGGL(k_min_partials, dim3(1), dim3(256), 0, st, grid, partial + kSumTail, cfl,
                       dt);
    return (int)hipGetLastError();
}

int launch_local_dt(int N, const double *vol, const double *lam, double cfl, double *dt,
                    hipStream_t st)
{
    const int grid = std::min(kRkBlocks, std::max(1, (N + kRkThreads - 1) / kRkThreads));
    hipLaunchKernelGGL(k_local_dt, dim3(grid), dim3(kRkThreads), 0, st, N, vol, lam, cfl, dt);
    return (int)hipGetLastError();
}

}  // namespace gpu
}  // namespace opf
