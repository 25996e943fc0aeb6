/*
 * oracle.h -- sequential FP64 reference of the edge-flux hot path.
 *
 * TEST INFRASTRUCTURE: used only by the test suite, the smoke check and the
 * CPU baseline of the benchmark.  Host arrays, SoA (component c of element k
 * at a[c*count + k]), 0-based row-major edge->node pairs.
 */
#ifndef ORACLE_H
#define ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ERANGE = -2, ORC_ENOMEM = -7 };

/* alpha_k of the 5-stage scheme, k = 0..4 */
double orc_rk_alpha(int k);

/* Flux of one edge from q_i to q_j with weight n (F added to i, subtracted from j). */
void orc_flux(const double qi[6], const double qj[6], const double n[3], double gamma,
              double F[6]);

/* res[6N] += sum over edges of +F at the first node and -F at the second.
 * S[6N] (optional) += |F| at both nodes: the scale of each residual entry. */
int orc_residual(int64_t N, int64_t E, const int32_t *e2n, const double *q, const double *w,
                 double gamma, double *res, double *S);

/* ss[v] = sum_i res[v,i]^2 (compensated); q = q0 - alpha_dt*res/vol; res = 0. */
int orc_rk_stage(int64_t N, const double *q0, double *res, const double *vol, double alpha_dt,
                 double *q, double ss[6]);

/* One 5-stage iteration in place on q0; ss[6k + v] is stage k's sum of squares. */
int orc_rk_iteration(int64_t N, int64_t E, const int32_t *e2n, double *q0, const double *w,
                     const double *vol, double gamma, double dt, double ss[30]);

/* lam_sum[N] += sum over incident edges of lambda_e. */
int orc_spectral_radius(int64_t N, int64_t E, const int32_t *e2n, const double *q,
                        const double *w, double gamma, double *lam_sum);

/* dt[N] = cfl * vol_i / sum_{e at i} lambda_e: the local time step of each node. */
int orc_local_dt(int64_t N, int64_t E, const int32_t *e2n, const double *q, const double *w,
                 const double *vol, double gamma, double cfl, double *dt);

/* As orc_rk_stage with a time step per node: q = q0 - alpha*dt_i*res/vol. */
int orc_rk_stage_local(int64_t N, const double *q0, double *res, const double *vol,
                       const double *dt, double alpha, double *q, double ss[6]);

/* One 5-stage iteration in place on q0 with the local time steps dt[N]. */
int orc_rk_iteration_local(int64_t N, int64_t E, const int32_t *e2n, double *q0, const double *w,
                           const double *vol, double gamma, const double *dt, double ss[30]);

/* cfl * min_i vol_i / sum_{e at i} lambda_e; negative on error. */
double orc_dt(int64_t N, int64_t E, const int32_t *e2n, const double *q, const double *w,
              const double *vol, double gamma, double cfl);

/* Green-Gauss sums over the median-dual cells: for each edge, +1/2 (q_i + q_j)
 * n_e is added to node i and subtracted from node j.  G holds 18 components
 * per node, (v, d) at G[(3v + d) N + k]; the nodal gradient is G / vol. */
int orc_gradient(int64_t N, int64_t E, const int32_t *e2n, const double *q, const double *w,
                 double *G);

/* Second-order residual: the edge flux of the reconstructed states
 * q_L = q_i + 1/2 (G_i / vol_i) . d_e and q_R = q_j - 1/2 (G_j / vol_j) . d_e,
 * d_e = x_j - x_i (dx[3E]); res[6N] += F(q_L, q_R, n_e) at i, -= at j. */
int orc_residual2(int64_t N, int64_t E, const int32_t *e2n, const double *q, const double *G,
                  const double *vol, const double *w, const double *dx, double gamma,
                  double *res);

/* Median-dual geometry of a tetrahedral mesh: for every tet (t2n[4t..4t+3],
 * positively oriented) and each of its six local edges, in the order (0,1),
 * (0,2), (0,3), (1,2), (1,3), (2,3) with global edge t2e[6t + k], the area
 * vector of the dual face inside the tet is added to w (3E, oriented from the
 * edge's first to its second node, e2n), and a quarter of the tet's volume to
 * vol (N) at each vertex.  xyz is 3N; period > 0 unwraps every vertex to the
 * image nearest vertex 0 in a periodic box of that side. */
int orc_geometry(int64_t N, int64_t E, int64_t T, const int32_t *e2n, const int32_t *t2n,
                 const int32_t *t2e, const double *xyz, double period, double *w, double *vol);

/* Reverse of orc_geometry: xbar (3N) += (dw/dx)^T wbar + (dvol/dx)^T volbar. */
int orc_geometry_adjoint(int64_t N, int64_t E, int64_t T, const int32_t *e2n, const int32_t *t2n,
                         const int32_t *t2e, const double *xyz, double period,
                         const double *wbar, const double *volbar, double *xbar);

/* jv[6N] = J (dq, dw): the residual's directional derivative (dual numbers). */
int orc_jvp(int64_t N, int64_t E, const int32_t *e2n, const double *q, const double *w,
            double gamma, const double *dq, const double *dw, double *jv);

/* Exact 6x15 Jacobian of one edge's flux w.r.t. (q_i, q_j, n), row-major. */
int orc_edge_jacobian(const double qi[6], const double qj[6], const double n[3], double gamma,
                      double F[6], double J[6 * 15]);

/* qbar[6N] = sum_e J_q^T (rbar_i - rbar_j); wbar[3E] = J_n^T (rbar_i - rbar_j). */
int orc_adjoint(int64_t N, int64_t E, const int32_t *e2n, const double *q, const double *w,
                double gamma, const double *rbar, double *qbar, double *wbar);

#ifdef __cplusplus
}
#endif
#endif
