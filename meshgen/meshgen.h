/*
 * meshgen.h -- seeded synthetic periodic tetrahedral meshes and states.
 *
 * Shared input source for the oracle and the GPU path.  Holds no arithmetic
 * of the edge-flux method itself.  All arrays are caller-allocated host memory.
 */
#ifndef MESHGEN_H
#define MESHGEN_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MG_PURPOSE_JITTER = 1,
    MG_PURPOSE_PERM = 2,
    MG_PURPOSE_LAYERS = 3,
    MG_PURPOSE_STATE = 4
};

typedef struct {
    int32_t n;          /* nodes per axis, >= 3 (multiple of 4 for split 1) */
    int32_t split;      /* 0: Kuhn 6-tet cubes; 1: layered 5/6 mix */
    int32_t permute;    /* 1: seeded random node labels; 0: generator order */
    int32_t pad;
    double jitter;      /* node jitter amplitude as a fraction of h, in [0, 0.5) */
    uint64_t mesh_seed; /* seeds jitter, relabelling and layer choice */
} mg_params;

/* N = n^3 nodes, E edges, T tets.  Returns 0, or -1 for invalid parameters. */
int mg_sizes(const mg_params *p, int64_t *N, int64_t *E, int64_t *T);

/* Builds the mesh.
 *   e2n  [2E]  edge->node map, row-major pairs (first, second), user labels;
 *              edges listed in lexicographic order of generator ids (a < b),
 *              first endpoint = relabelled a.
 *   w    [3E]  SoA median-dual edge weights, component d of edge e at d*E+e,
 *              pointing from the first endpoint to the second.
 *   vol  [N]   median-dual volumes (user labels).
 *   xyz  [3N]  SoA node positions (user labels, not wrapped after jitter).
 *   perm [N]   perm[g] = user label of generator node g.
 *   stats[3]   (inverted tets, 6-tet cubes, tets); may be NULL.
 * Returns 0, -1 (invalid parameters), -2 (out of memory), -4 (internal). */
int mg_build(const mg_params *p, int32_t *e2n, double *w, double *vol, double *xyz,
             int32_t *perm, int64_t *stats);

/* Tets [4T] as user labels, positively oriented on the lattice template. */
int mg_tets(const mg_params *p, const int32_t *perm, int32_t *tets);

/* Initial state q [6N] SoA (rho, rho u, rho v, rho w, rho E, rho phi) drawn per
 * generator node: rho, p ~ U(0.9,1.1); u, v, w ~ U(-0.3,0.3); phi ~ U(0,1).
 * perm may be NULL (identity). */
int mg_state(int64_t N, const int32_t *perm, uint64_t seed, double gamma, double *q);

/* Six median-dual edge weights of one tet x[4][3] (edges 01,02,03,12,13,23)
 * and its signed volume. */
int mg_tet_dual(const double x[12], double nvec[18], double *vol);

/* Edge ids (row of e2n) of the six local edges of each tet, in the order
 * (0,1) (0,2) (0,3) (1,2) (1,3) (2,3): out is T x 6.  Connectivity only.
 * Returns 0, -1 when a tet edge is missing from e2n, -7 on allocation failure. */
int mg_tet_edges(int64_t N, int64_t E, const int32_t *e2n, int64_t T, const int32_t *tets,
                 int32_t *out);

uint64_t mg_stream(uint64_t seed, uint64_t purpose);
void mg_uniform(uint64_t seed, uint64_t purpose, int64_t count, double lo, double hi,
                double *out);
void mg_normal(uint64_t seed, uint64_t purpose, int64_t count, double *out);

#ifdef __cplusplus
}
#endif
#endif
