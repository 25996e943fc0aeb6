/*
 * oracle.c -- plain sequential FP64 reference of the edge-flux hot path.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the GPU library, and the GPU library never
 * calls it.
 *
 * What it follows (the paper gives the loop semantics, not the numerics):
 *  - Sec. 3.2: a single-threaded sequential back-end is the reference every
 *    parallel build must reproduce; here it is a plain loop over edges in
 *    input order, no plan, no threads, no blocking.
 *  - Sec. 3.1 (the op_par_loop example): OP_INC through a map is a sequential
 *    sum over the set elements; an edge loop reads its two nodes through the
 *    edge->node map and increments both.
 *  - Sec. 2: time marching with a 5-stage Runge-Kutta scheme.
 *  - The flux itself is not in the paper.  The workload defines it as
 *      F_e = 1/2 (f(q_i) + f(q_j)).n_e - 1/2 lambda_e (q_j - q_i),
 *      lambda_e = |u_avg.n_e| + c_avg |n_e|,
 *    with +F_e added to res_i and -F_e to res_j (Euler flux of the
 *    conservative state rho, rho u, rho v, rho w, rho E, rho phi, ideal gas).
 *
 * Readings taken where the definition is silent (each one is listed in the
 * design notes of the repository):
 *  - u_avg and c_avg are arithmetic means of the nodal velocity and sound speed;
 *  - the passive scalar is carried as rho*phi with flux rho*phi * (u.n);
 *  - the explicit update is q = q0 - alpha_k dt res/vol (the residual is the
 *    net outflow, so the sign must be negative for the scheme to be stable);
 *  - stage coefficients alpha = (1/4, 1/6, 3/8, 1/2, 1);
 *  - the residual norm is per variable, sum over nodes of res^2 (compensated);
 *  - d|x|/dx = +1 at x = +0.
 *
 * Arrays are host memory in SoA layout: component c of element k at
 * a[c * count + k].  Maps are row-major pairs e2n[2e], e2n[2e+1], 0-based.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static const double RK_ALPHA[5] = {1.0 / 4.0, 1.0 / 6.0, 3.0 / 8.0, 1.0 / 2.0, 1.0};

double orc_rk_alpha(int k) { return (k >= 0 && k < 5) ? RK_ALPHA[k] : 0.0; }

/* ---------------------------------------------------------- plain FP64 -- */

typedef struct {
    double u[3], p, c;
} prim;

static void node_prim(const double q[6], double gamma, prim *s)
{
    double rho = q[0];
    s->u[0] = q[1] / rho;
    s->u[1] = q[2] / rho;
    s->u[2] = q[3] / rho;
    s->p = (gamma - 1.0) * (q[4] - 0.5 * (q[1] * s->u[0] + q[2] * s->u[1] + q[3] * s->u[2]));
    s->c = sqrt(gamma * s->p / rho);
}

/* f(q).n for one node, given its primitives. */
static void normal_flux(const double q[6], const prim *s, const double n[3], double f[6])
{
    double U = s->u[0] * n[0] + s->u[1] * n[1] + s->u[2] * n[2];
    f[0] = q[0] * U;
    f[1] = q[1] * U + s->p * n[0];
    f[2] = q[2] * U + s->p * n[1];
    f[3] = q[3] * U + s->p * n[2];
    f[4] = (q[4] + s->p) * U;
    f[5] = q[5] * U;
}

static void edge_flux(const double qi[6], const prim *si, const double qj[6], const prim *sj,
                      const double n[3], double F[6])
{
    double fi[6], fj[6];
    normal_flux(qi, si, n, fi);
    normal_flux(qj, sj, n, fj);
    double Ui = si->u[0] * n[0] + si->u[1] * n[1] + si->u[2] * n[2];
    double Uj = sj->u[0] * n[0] + sj->u[1] * n[1] + sj->u[2] * n[2];
    double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    double lam = fabs(0.5 * (Ui + Uj)) + 0.5 * (si->c + sj->c) * nn;
    for (int v = 0; v < 6; ++v) F[v] = 0.5 * (fi[v] + fj[v]) - 0.5 * lam * (qj[v] - qi[v]);
}

void orc_flux(const double qi[6], const double qj[6], const double n[3], double gamma,
              double F[6])
{
    prim si, sj;
    node_prim(qi, gamma, &si);
    node_prim(qj, gamma, &sj);
    edge_flux(qi, &si, qj, &sj, n, F);
}

static void gather6(const double *q, int64_t N, int64_t i, double out[6])
{
    for (int v = 0; v < 6; ++v) out[v] = q[(int64_t)v * N + i];
}

static int check_map(int64_t N, int64_t E, const int32_t *e2n)
{
    for (int64_t e = 0; e < 2 * E; ++e)
        if (e2n[e] < 0 || e2n[e] >= N) return ORC_ERANGE;
    return 0;
}

int orc_residual(int64_t N, int64_t E, const int32_t *e2n, const double *q, const double *w,
                 double gamma, double *res, double *S)
{
    if (N <= 0 || E < 0) return ORC_EINVAL;
    if (check_map(N, E, e2n)) return ORC_ERANGE;
    prim *P = malloc((size_t)N * sizeof(prim));
    if (!P) return ORC_ENOMEM;
    for (int64_t i = 0; i < N; ++i) {
        double qi[6];
        gather6(q, N, i, qi);
        node_prim(qi, gamma, &P[i]);
    }
    for (int64_t e = 0; e < E; ++e) {
        int64_t i = e2n[2 * e], j = e2n[2 * e + 1];
        double qi[6], qj[6], n[3], F[6];
        gather6(q, N, i, qi);
        gather6(q, N, j, qj);
        for (int d = 0; d < 3; ++d) n[d] = w[(int64_t)d * E + e];
        edge_flux(qi, &P[i], qj, &P[j], n, F);
        for (int v = 0; v < 6; ++v) {
            res[(int64_t)v * N + i] += F[v];
            res[(int64_t)v * N + j] -= F[v];
            if (S) {
                S[(int64_t)v * N + i] += fabs(F[v]);
                S[(int64_t)v * N + j] += fabs(F[v]);
            }
        }
    }
    free(P);
    return 0;
}

/* Gradient and second-order flux.  The paper names the loops (a gradient
 * accumulation over edges and the dominant viscous edge flux, Sec. 4's loop
 * tables) but not their numerics.  Readings: the gradient is the Green-Gauss
 * sum over each median-dual cell with the face value taken as the mean of the
 * two end states; the second-order flux applies the first-order edge flux to
 * states reconstructed linearly, without a limiter, to the edge midpoint. */
int orc_gradient(int64_t N, int64_t E, const int32_t *e2n, const double *q, const double *w,
                 double *G)
{
    if (N <= 0 || E < 0) return ORC_EINVAL;
    if (check_map(N, E, e2n)) return ORC_ERANGE;
    for (int64_t e = 0; e < E; ++e) {
        int64_t i = e2n[2 * e], j = e2n[2 * e + 1];
        for (int v = 0; v < 6; ++v) {
            double face = 0.5 * (q[(int64_t)v * N + i] + q[(int64_t)v * N + j]);
            for (int d = 0; d < 3; ++d) {
                double g = face * w[(int64_t)d * E + e];
                G[(int64_t)(3 * v + d) * N + i] += g;
                G[(int64_t)(3 * v + d) * N + j] -= g;
            }
        }
    }
    return 0;
}

int orc_residual2(int64_t N, int64_t E, const int32_t *e2n, const double *q, const double *G,
                  const double *vol, const double *w, const double *dx, double gamma,
                  double *res)
{
    if (N <= 0 || E < 0) return ORC_EINVAL;
    if (check_map(N, E, e2n)) return ORC_ERANGE;
    for (int64_t e = 0; e < E; ++e) {
        int64_t i = e2n[2 * e], j = e2n[2 * e + 1];
        double qL[6], qR[6], n[3], d[3], F[6];
        for (int k = 0; k < 3; ++k) {
            n[k] = w[(int64_t)k * E + e];
            d[k] = dx[(int64_t)k * E + e];
        }
        for (int v = 0; v < 6; ++v) {
            double si = 0.0, sj = 0.0;
            for (int k = 0; k < 3; ++k) {
                si += G[(int64_t)(3 * v + k) * N + i] / vol[i] * d[k];
                sj += G[(int64_t)(3 * v + k) * N + j] / vol[j] * d[k];
            }
            qL[v] = q[(int64_t)v * N + i] + 0.5 * si;
            qR[v] = q[(int64_t)v * N + j] - 0.5 * sj;
        }
        orc_flux(qL, qR, n, gamma, F);
        for (int v = 0; v < 6; ++v) {
            res[(int64_t)v * N + i] += F[v];
            res[(int64_t)v * N + j] -= F[v];
        }
    }
    return 0;
}

/* Median-dual geometry.  Inside a tet (p, q, r, s), the dual face between the
 * cells of p and q joins the edge midpoint, the centroids of faces pqr and
 * pqs and the tet centroid; its area vector (half the cross product of the
 * quadrilateral's diagonals) is (r + s - p - q) x (s - r) / 24, pointing from
 * p to q when (p, q, r, s) has the orientation of the tet.  For local edge
 * (a, b) the completing pair (r, s) is chosen so that (a, b, r, s) is an even
 * permutation of (0, 1, 2, 3).  Each vertex owns a quarter of the tet. */
static const int GEO_EDGE[6][4] = {{0, 1, 2, 3}, {0, 2, 3, 1}, {0, 3, 1, 2},
                                   {1, 2, 0, 3}, {1, 3, 2, 0}, {2, 3, 0, 1}};

static void cross(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* The tet's vertex positions, unwrapped to the images nearest vertex 0. */
static void tet_positions(int64_t N, const int32_t *t2n, int64_t t, const double *xyz,
                          double period, double x[4][3])
{
    for (int v = 0; v < 4; ++v)
        for (int d = 0; d < 3; ++d) x[v][d] = xyz[(int64_t)d * N + t2n[4 * t + v]];
    if (period > 0.0)
        for (int v = 1; v < 4; ++v)
            for (int d = 0; d < 3; ++d)
                x[v][d] -= period * round((x[v][d] - x[0][d]) / period);
}

/* +1 when global edge g runs from local vertex a to local vertex b, -1 when
 * it runs the other way, 0 when it is not that edge. */
static double edge_sign(const int32_t *e2n, const int32_t *t2n, int64_t t, int64_t g, int a, int b)
{
    int32_t na = t2n[4 * t + a], nb = t2n[4 * t + b];
    if (e2n[2 * g] == na && e2n[2 * g + 1] == nb) return 1.0;
    if (e2n[2 * g] == nb && e2n[2 * g + 1] == na) return -1.0;
    return 0.0;
}

static int check_tets(int64_t N, int64_t E, int64_t T, const int32_t *t2n, const int32_t *t2e)
{
    for (int64_t k = 0; k < 4 * T; ++k)
        if (t2n[k] < 0 || t2n[k] >= N) return ORC_ERANGE;
    for (int64_t k = 0; k < 6 * T; ++k)
        if (t2e[k] < 0 || t2e[k] >= E) return ORC_ERANGE;
    return 0;
}

int orc_geometry(int64_t N, int64_t E, int64_t T, const int32_t *e2n, const int32_t *t2n,
                 const int32_t *t2e, const double *xyz, double period, double *w, double *vol)
{
    if (N <= 0 || E <= 0 || T < 0) return ORC_EINVAL;
    if (check_map(N, E, e2n) || check_tets(N, E, T, t2n, t2e)) return ORC_ERANGE;
    for (int64_t t = 0; t < T; ++t) {
        double x[4][3];
        tet_positions(N, t2n, t, xyz, period, x);
        for (int k = 0; k < 6; ++k) {
            const int *L = GEO_EDGE[k];
            double a[3], b[3], c[3];
            for (int d = 0; d < 3; ++d) {
                a[d] = x[L[2]][d] + x[L[3]][d] - x[L[0]][d] - x[L[1]][d];
                b[d] = x[L[3]][d] - x[L[2]][d];
            }
            cross(a, b, c);
            int64_t g = t2e[6 * t + k];
            double sg = edge_sign(e2n, t2n, t, g, L[0], L[1]);
            if (sg == 0.0) return ORC_EINVAL;
            for (int d = 0; d < 3; ++d) w[(int64_t)d * E + g] += sg * c[d] / 24.0;
        }
        double e1[3], e2[3], e3[3], c[3];
        for (int d = 0; d < 3; ++d) {
            e1[d] = x[1][d] - x[0][d];
            e2[d] = x[2][d] - x[0][d];
            e3[d] = x[3][d] - x[0][d];
        }
        cross(e2, e3, c);
        double V = (e1[0] * c[0] + e1[1] * c[1] + e1[2] * c[2]) / 6.0;
        for (int v = 0; v < 4; ++v) vol[t2n[4 * t + v]] += 0.25 * V;
    }
    return 0;
}

int orc_geometry_adjoint(int64_t N, int64_t E, int64_t T, const int32_t *e2n, const int32_t *t2n,
                         const int32_t *t2e, const double *xyz, double period,
                         const double *wbar, const double *volbar, double *xbar)
{
    if (N <= 0 || E <= 0 || T < 0) return ORC_EINVAL;
    if (check_map(N, E, e2n) || check_tets(N, E, T, t2n, t2e)) return ORC_ERANGE;
    for (int64_t t = 0; t < T; ++t) {
        double x[4][3], xb[4][3] = {{0}};
        tet_positions(N, t2n, t, xyz, period, x);
        /* c = a x b / 24: abar = b x cbar / 24, bbar = cbar x a / 24 */
        for (int k = 0; k < 6; ++k) {
            const int *L = GEO_EDGE[k];
            int64_t g = t2e[6 * t + k];
            double sg = edge_sign(e2n, t2n, t, g, L[0], L[1]);
            if (sg == 0.0) return ORC_EINVAL;
            double a[3], b[3], cb[3], ab[3], bb[3];
            for (int d = 0; d < 3; ++d) {
                a[d] = x[L[2]][d] + x[L[3]][d] - x[L[0]][d] - x[L[1]][d];
                b[d] = x[L[3]][d] - x[L[2]][d];
                cb[d] = sg * wbar[(int64_t)d * E + g] / 24.0;
            }
            cross(b, cb, ab);
            cross(cb, a, bb);
            for (int d = 0; d < 3; ++d) {
                xb[L[0]][d] -= ab[d];
                xb[L[1]][d] -= ab[d];
                xb[L[2]][d] += ab[d] - bb[d];
                xb[L[3]][d] += ab[d] + bb[d];
            }
        }
        /* V = e1 . (e2 x e3) / 6, e_k = x_k - x_0 */
        double Vb = 0.0;
        for (int v = 0; v < 4; ++v) Vb += 0.25 * volbar[t2n[4 * t + v]];
        double e1[3], e2[3], e3[3], c1[3], c2[3], c3[3];
        for (int d = 0; d < 3; ++d) {
            e1[d] = x[1][d] - x[0][d];
            e2[d] = x[2][d] - x[0][d];
            e3[d] = x[3][d] - x[0][d];
        }
        cross(e2, e3, c1);
        cross(e3, e1, c2);
        cross(e1, e2, c3);
        for (int d = 0; d < 3; ++d) {
            xb[1][d] += Vb * c1[d] / 6.0;
            xb[2][d] += Vb * c2[d] / 6.0;
            xb[3][d] += Vb * c3[d] / 6.0;
            xb[0][d] -= Vb * (c1[d] + c2[d] + c3[d]) / 6.0;
        }
        for (int v = 0; v < 4; ++v)
            for (int d = 0; d < 3; ++d) xbar[(int64_t)d * N + t2n[4 * t + v]] += xb[v][d];
    }
    return 0;
}

/* Neumaier's compensated summation. */
typedef struct {
    double s, c;
} ksum;

static void ksum_add(ksum *k, double x)
{
    double t = k->s + x;
    if (fabs(k->s) >= fabs(x))
        k->c += (k->s - t) + x;
    else
        k->c += (x - t) + k->s;
    k->s = t;
}

int orc_rk_stage(int64_t N, const double *q0, double *res, const double *vol, double alpha_dt,
                 double *q, double ss[6])
{
    if (N <= 0) return ORC_EINVAL;
    for (int v = 0; v < 6; ++v) {
        ksum k = {0.0, 0.0};
        for (int64_t i = 0; i < N; ++i) {
            double r = res[(int64_t)v * N + i];
            ksum_add(&k, r * r);
            q[(int64_t)v * N + i] = q0[(int64_t)v * N + i] - alpha_dt * r / vol[i];
            res[(int64_t)v * N + i] = 0.0;
        }
        ss[v] = k.s + k.c;
    }
    return 0;
}

/* Local time stepping: each node advances with its own stable step, the
 * global step of Sec. 2's explicit scheme taken node by node; the stage
 * coefficients stay those of the 5-stage scheme. */
int orc_rk_stage_local(int64_t N, const double *q0, double *res, const double *vol,
                       const double *dt, double alpha, double *q, double ss[6])
{
    if (N <= 0) return ORC_EINVAL;
    for (int v = 0; v < 6; ++v) {
        ksum k = {0.0, 0.0};
        for (int64_t i = 0; i < N; ++i) {
            double r = res[(int64_t)v * N + i];
            ksum_add(&k, r * r);
            q[(int64_t)v * N + i] = q0[(int64_t)v * N + i] - alpha * dt[i] * r / vol[i];
            res[(int64_t)v * N + i] = 0.0;
        }
        ss[v] = k.s + k.c;
    }
    return 0;
}

int orc_rk_iteration_local(int64_t N, int64_t E, const int32_t *e2n, double *q0, const double *w,
                           const double *vol, double gamma, const double *dt, double ss[30])
{
    double *res = calloc((size_t)N * 6, sizeof(double));
    double *q = malloc((size_t)N * 6 * sizeof(double));
    if (!res || !q) {
        free(res);
        free(q);
        return ORC_ENOMEM;
    }
    memcpy(q, q0, (size_t)N * 6 * sizeof(double));
    int rc = 0;
    for (int k = 0; k < 5 && !rc; ++k) {
        rc = orc_residual(N, E, e2n, q, w, gamma, res, NULL);
        if (!rc) rc = orc_rk_stage_local(N, q0, res, vol, dt, RK_ALPHA[k], q, ss + 6 * k);
    }
    if (!rc) memcpy(q0, q, (size_t)N * 6 * sizeof(double));
    free(res);
    free(q);
    return rc;
}

int orc_rk_iteration(int64_t N, int64_t E, const int32_t *e2n, double *q0, const double *w,
                     const double *vol, double gamma, double dt, double ss[30])
{
    double *res = calloc((size_t)N * 6, sizeof(double));
    double *q = malloc((size_t)N * 6 * sizeof(double));
    if (!res || !q) {
        free(res);
        free(q);
        return ORC_ENOMEM;
    }
    memcpy(q, q0, (size_t)N * 6 * sizeof(double));
    int rc = 0;
    for (int k = 0; k < 5 && !rc; ++k) {
        rc = orc_residual(N, E, e2n, q, w, gamma, res, NULL);
        if (!rc) rc = orc_rk_stage(N, q0, res, vol, RK_ALPHA[k] * dt, q, ss + 6 * k);
    }
    if (!rc) memcpy(q0, q, (size_t)N * 6 * sizeof(double));
    free(res);
    free(q);
    return rc;
}

int orc_spectral_radius(int64_t N, int64_t E, const int32_t *e2n, const double *q,
                        const double *w, double gamma, double *lam_sum)
{
    if (N <= 0 || E < 0) return ORC_EINVAL;
    if (check_map(N, E, e2n)) return ORC_ERANGE;
    for (int64_t e = 0; e < E; ++e) {
        int64_t i = e2n[2 * e], j = e2n[2 * e + 1];
        double qi[6], qj[6], n[3];
        prim si, sj;
        gather6(q, N, i, qi);
        gather6(q, N, j, qj);
        node_prim(qi, gamma, &si);
        node_prim(qj, gamma, &sj);
        for (int d = 0; d < 3; ++d) n[d] = w[(int64_t)d * E + e];
        double Ui = si.u[0] * n[0] + si.u[1] * n[1] + si.u[2] * n[2];
        double Uj = sj.u[0] * n[0] + sj.u[1] * n[1] + sj.u[2] * n[2];
        double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        double lam = fabs(0.5 * (Ui + Uj)) + 0.5 * (si.c + sj.c) * nn;
        lam_sum[i] += lam;
        lam_sum[j] += lam;
    }
    return 0;
}

int orc_local_dt(int64_t N, int64_t E, const int32_t *e2n, const double *q, const double *w,
                 const double *vol, double gamma, double cfl, double *dt)
{
    double *ls = calloc((size_t)N, sizeof(double));
    if (!ls) return ORC_ENOMEM;
    int rc = orc_spectral_radius(N, E, e2n, q, w, gamma, ls);
    if (!rc)
        for (int64_t i = 0; i < N; ++i) dt[i] = cfl * vol[i] / ls[i];
    free(ls);
    return rc;
}

double orc_dt(int64_t N, int64_t E, const int32_t *e2n, const double *q, const double *w,
              const double *vol, double gamma, double cfl)
{
    double *ls = calloc((size_t)N, sizeof(double));
    if (!ls) return -1.0;
    if (orc_spectral_radius(N, E, e2n, q, w, gamma, ls)) {
        free(ls);
        return -1.0;
    }
    double dt = INFINITY;
    for (int64_t i = 0; i < N; ++i) {
        double t = vol[i] / ls[i];
        if (t < dt) dt = t;
    }
    free(ls);
    return cfl * dt;
}

/* ------------------------------------------------------- dual numbers -- */

/* Forward-mode dual number with up to 15 tangent directions: value and
 * derivatives propagated by the chain rule, one elementary operation at a
 * time.  Only the first `nt` tangents are used. */
#define NT_MAX 15
typedef struct {
    double v, d[NT_MAX];
} dn;

static int nt;

static dn dconst(double x)
{
    dn r;
    r.v = x;
    for (int k = 0; k < NT_MAX; ++k) r.d[k] = 0.0;
    return r;
}
static dn dadd(dn a, dn b)
{
    dn r;
    r.v = a.v + b.v;
    for (int k = 0; k < nt; ++k) r.d[k] = a.d[k] + b.d[k];
    return r;
}
static dn dsub(dn a, dn b)
{
    dn r;
    r.v = a.v - b.v;
    for (int k = 0; k < nt; ++k) r.d[k] = a.d[k] - b.d[k];
    return r;
}
static dn dmul(dn a, dn b)
{
    dn r;
    r.v = a.v * b.v;
    for (int k = 0; k < nt; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
    return r;
}
static dn dscale(double s, dn a)
{
    dn r;
    r.v = s * a.v;
    for (int k = 0; k < nt; ++k) r.d[k] = s * a.d[k];
    return r;
}
static dn ddiv(dn a, dn b)
{
    dn r;
    r.v = a.v / b.v;
    for (int k = 0; k < nt; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) / b.v;
    return r;
}
static dn dsqrt(dn a)
{
    dn r;
    r.v = sqrt(a.v);
    for (int k = 0; k < nt; ++k) r.d[k] = a.d[k] / (2.0 * r.v);
    return r;
}
static dn dabs(dn a)
{
    double s = signbit(a.v) ? -1.0 : 1.0;
    return dscale(s, a);
}

/* Flux of one edge on dual numbers, the same formula as edge_flux(). */
static void dual_flux(const dn qi[6], const dn qj[6], const dn n[3], double gamma, dn F[6])
{
    const dn *qs[2] = {qi, qj};
    dn u[2][3], p[2], c[2], U[2], f[2][6];
    for (int s = 0; s < 2; ++s) {
        const dn *q = qs[s];
        for (int d = 0; d < 3; ++d) u[s][d] = ddiv(q[1 + d], q[0]);
        dn ke = dadd(dadd(dmul(q[1], u[s][0]), dmul(q[2], u[s][1])), dmul(q[3], u[s][2]));
        p[s] = dscale(gamma - 1.0, dsub(q[4], dscale(0.5, ke)));
        c[s] = dsqrt(ddiv(dscale(gamma, p[s]), q[0]));
        U[s] = dadd(dadd(dmul(u[s][0], n[0]), dmul(u[s][1], n[1])), dmul(u[s][2], n[2]));
        f[s][0] = dmul(q[0], U[s]);
        for (int d = 0; d < 3; ++d) f[s][1 + d] = dadd(dmul(q[1 + d], U[s]), dmul(p[s], n[d]));
        f[s][4] = dmul(dadd(q[4], p[s]), U[s]);
        f[s][5] = dmul(q[5], U[s]);
    }
    dn nn = dsqrt(dadd(dadd(dmul(n[0], n[0]), dmul(n[1], n[1])), dmul(n[2], n[2])));
    dn lam = dadd(dabs(dscale(0.5, dadd(U[0], U[1]))), dmul(dscale(0.5, dadd(c[0], c[1])), nn));
    for (int v = 0; v < 6; ++v)
        F[v] = dsub(dscale(0.5, dadd(f[0][v], f[1][v])), dmul(dscale(0.5, lam), dsub(qj[v], qi[v])));
}

int orc_jvp(int64_t N, int64_t E, const int32_t *e2n, const double *q, const double *w,
            double gamma, const double *dq, const double *dw, double *jv)
{
    if (N <= 0 || E < 0) return ORC_EINVAL;
    if (check_map(N, E, e2n)) return ORC_ERANGE;
    nt = 1;
    memset(jv, 0, (size_t)N * 6 * sizeof(double));
    for (int64_t e = 0; e < E; ++e) {
        int64_t i = e2n[2 * e], j = e2n[2 * e + 1];
        dn qi[6], qj[6], n[3], F[6];
        for (int v = 0; v < 6; ++v) {
            qi[v] = dconst(q[(int64_t)v * N + i]);
            qi[v].d[0] = dq ? dq[(int64_t)v * N + i] : 0.0;
            qj[v] = dconst(q[(int64_t)v * N + j]);
            qj[v].d[0] = dq ? dq[(int64_t)v * N + j] : 0.0;
        }
        for (int d = 0; d < 3; ++d) {
            n[d] = dconst(w[(int64_t)d * E + e]);
            n[d].d[0] = dw ? dw[(int64_t)d * E + e] : 0.0;
        }
        dual_flux(qi, qj, n, gamma, F);
        for (int v = 0; v < 6; ++v) {
            jv[(int64_t)v * N + i] += F[v].d[0];
            jv[(int64_t)v * N + j] -= F[v].d[0];
        }
    }
    return 0;
}

int orc_edge_jacobian(const double qi[6], const double qj[6], const double n[3], double gamma,
                      double F[6], double J[6 * 15])
{
    nt = 15;
    dn a[6], b[6], m[3], G[6];
    for (int v = 0; v < 6; ++v) {
        a[v] = dconst(qi[v]);
        a[v].d[v] = 1.0;
        b[v] = dconst(qj[v]);
        b[v].d[6 + v] = 1.0;
    }
    for (int d = 0; d < 3; ++d) {
        m[d] = dconst(n[d]);
        m[d].d[12 + d] = 1.0;
    }
    dual_flux(a, b, m, gamma, G);
    for (int v = 0; v < 6; ++v) {
        if (F) F[v] = G[v].v;
        for (int k = 0; k < 15; ++k) J[15 * v + k] = G[v].d[k];
    }
    return 0;
}

int orc_adjoint(int64_t N, int64_t E, const int32_t *e2n, const double *q, const double *w,
                double gamma, const double *rbar, double *qbar, double *wbar)
{
    if (N <= 0 || E < 0) return ORC_EINVAL;
    if (check_map(N, E, e2n)) return ORC_ERANGE;
    memset(qbar, 0, (size_t)N * 6 * sizeof(double));
    for (int64_t e = 0; e < E; ++e) {
        int64_t i = e2n[2 * e], j = e2n[2 * e + 1];
        double qi[6], qj[6], n[3], J[6 * 15], Fb[6];
        gather6(q, N, i, qi);
        gather6(q, N, j, qj);
        for (int d = 0; d < 3; ++d) n[d] = w[(int64_t)d * E + e];
        orc_edge_jacobian(qi, qj, n, gamma, NULL, J);
        /* res_i gets +F and res_j gets -F, so dL/dF = rbar_i - rbar_j */
        for (int v = 0; v < 6; ++v) Fb[v] = rbar[(int64_t)v * N + i] - rbar[(int64_t)v * N + j];
        for (int k = 0; k < 15; ++k) {
            double s = 0.0;
            for (int v = 0; v < 6; ++v) s += J[15 * v + k] * Fb[v];
            if (k < 6)
                qbar[(int64_t)k * N + i] += s;
            else if (k < 12)
                qbar[(int64_t)(k - 6) * N + j] += s;
            else
                wbar[(int64_t)(k - 12) * E + e] = s;
        }
    }
    return 0;
}
