/*
 * meshgen.c -- seeded synthetic inputs for the edge-flux loop.
 *
 * Builds periodic tetrahedral meshes of the unit box shaped like the
 * unstructured turbomachinery meshes the paper measures on (Sec. 4: node and
 * edge sets, an edge->node map of arity 2, three direct values per edge),
 * together with the initial node state and random vectors used by the
 * derivative checks.  This module is shared by the oracle and by the GPU
 * path as their common input source; it holds no flux, update or reduction
 * arithmetic of the method -- only geometry (median-dual edge weights and
 * dual volumes), random numbers and the primitive->conservative conversion of
 * the initial state.
 *
 * Random numbers: SplitMix64 (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014), uniform doubles as
 * (x >> 11) * 2^-53, normals by the Box-Muller transform.  Every purpose
 * draws from its own stream derived from (seed, purpose).
 *
 * Mesh families
 *   split 0: every cube cell cut into the 6 Kuhn tetrahedra around the body
 *            diagonal from its (0,0,0) corner; E = 7 N.
 *   split 1: layered 5/6 mix.  Exactly n/2 of the n z-layers (chosen by seed)
 *            use 6-tet cubes, the others 5-tet cubes; face diagonals agree
 *            across every shared face, so the mesh is conforming and periodic
 *            (n a multiple of 4, so that the n/2 parity flips of the
 *            horizontal faces close up).  E = 6.5 N, T = 5.5 n^3.
 * Orientation of every tetrahedron is taken from its integer lattice
 * template, never from jittered positions, so the dual control volumes close
 * exactly even where jitter inverts a tetrahedron.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "meshgen.h"

/* ---------------------------------------------------------------- RNG -- */

static inline uint64_t sm_next(uint64_t *s)
{
    uint64_t z = (*s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t mg_stream(uint64_t seed, uint64_t purpose)
{
    uint64_t s = seed ^ (purpose * 0xD1B54A32D192ED03ULL);
    (void)sm_next(&s);
    return s;
}

static inline double sm_uniform(uint64_t *s) /* [0, 1) */
{
    return (double)(sm_next(s) >> 11) * 0x1.0p-53;
}

static inline uint64_t sm_below(uint64_t *s, uint64_t bound) /* [0, bound) */
{
    return (uint64_t)(((unsigned __int128)sm_next(s) * bound) >> 64);
}

void mg_uniform(uint64_t seed, uint64_t purpose, int64_t count, double lo, double hi,
                double *out)
{
    uint64_t s = mg_stream(seed, purpose);
    for (int64_t i = 0; i < count; ++i) out[i] = lo + (hi - lo) * sm_uniform(&s);
}

void mg_normal(uint64_t seed, uint64_t purpose, int64_t count, double *out)
{
    uint64_t s = mg_stream(seed, purpose);
    const double two_pi = 6.283185307179586476925286766559;
    for (int64_t i = 0; i < count; i += 2) {
        double u1 = sm_uniform(&s), u2 = sm_uniform(&s);
        double r = sqrt(-2.0 * log(1.0 - u1));
        out[i] = r * cos(two_pi * u2);
        if (i + 1 < count) out[i + 1] = r * sin(two_pi * u2);
    }
}

/* ----------------------------------------------------- tet dual weights -- */

/* For an edge (p,q) of a positively oriented tet (v0,v1,v2,v3), the other two
 * vertices (r,s) are taken so that (p,q,r,s) is an even permutation. */
static const int TET_EDGE[6][4] = {
    {0, 1, 2, 3}, {0, 2, 3, 1}, {0, 3, 1, 2}, {1, 2, 0, 3}, {1, 3, 2, 0}, {2, 3, 0, 1}};

static inline void cross3(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* Median-dual face of edge (p,q) inside one tet: the quadrilateral through the
 * edge midpoint, the two face centroids (pqr), (pqs) and the tet centroid.  Its
 * area vector is (x_r + x_s - x_p - x_q) x (x_s - x_r) / 24 and points from p
 * to q.  Also returns the signed tet volume. */
int mg_tet_dual(const double x[12], double nvec[18], double *vol)
{
    for (int e = 0; e < 6; ++e) {
        const double *p = x + 3 * TET_EDGE[e][0], *q = x + 3 * TET_EDGE[e][1];
        const double *r = x + 3 * TET_EDGE[e][2], *s = x + 3 * TET_EDGE[e][3];
        double a[3], b[3], c[3];
        for (int d = 0; d < 3; ++d) {
            a[d] = r[d] + s[d] - p[d] - q[d];
            b[d] = s[d] - r[d];
        }
        cross3(a, b, c);
        for (int d = 0; d < 3; ++d) nvec[3 * e + d] = c[d] / 24.0;
    }
    double e1[3], e2[3], e3[3], c[3];
    for (int d = 0; d < 3; ++d) {
        e1[d] = x[3 + d] - x[d];
        e2[d] = x[6 + d] - x[d];
        e3[d] = x[9 + d] - x[d];
    }
    cross3(e2, e3, c);
    *vol = (e1[0] * c[0] + e1[1] * c[1] + e1[2] * c[2]) / 6.0;
    return 0;
}

/* --------------------------------------------------------- lattice mesh -- */

typedef struct {
    int32_t n;
    int32_t split;
    int32_t *six;   /* per z-layer: 1 = 6-tet layer (split 1) */
    int32_t *zpar;  /* per z-plane: diagonal parity of horizontal faces */
    int32_t *alpha; /* per z-layer: seeded bit of the 6-tet corner choice */
} lattice;

static inline int64_t gid(const lattice *L, int64_t i, int64_t j, int64_t k)
{
    int64_t n = L->n;
    return (i % n) + n * ((j % n) + n * (k % n));
}

static int lattice_init(lattice *L, const mg_params *P)
{
    memset(L, 0, sizeof *L);
    L->n = P->n;
    L->split = P->split;
    if (P->n < 3) return -1;
    if (P->split != 0 && P->split != 1) return -1;
    if (P->split == 1 && (P->n % 4) != 0) return -1;
    if (P->split == 1) {
        int n = P->n;
        L->six = calloc((size_t)n, sizeof(int32_t));
        L->zpar = calloc((size_t)n + 1, sizeof(int32_t));
        L->alpha = calloc((size_t)n, sizeof(int32_t));
        int32_t *order = malloc((size_t)n * sizeof(int32_t));
        if (!L->six || !L->zpar || !L->alpha || !order) {
            free(order);
            return -2;
        }
        uint64_t s = mg_stream(P->mesh_seed, MG_PURPOSE_LAYERS);
        for (int k = 0; k < n; ++k) order[k] = k;
        for (int k = n - 1; k > 0; --k) { /* Fisher-Yates */
            int j = (int)sm_below(&s, (uint64_t)k + 1);
            int32_t t = order[k];
            order[k] = order[j];
            order[j] = t;
        }
        for (int k = 0; k < n / 2; ++k) L->six[order[k]] = 1;
        L->zpar[0] = (int32_t)(sm_next(&s) >> 63);
        for (int k = 0; k < n; ++k) {
            L->alpha[k] = (int32_t)(sm_next(&s) >> 63);
            L->zpar[k + 1] = L->six[k] ? 1 - L->zpar[k] : L->zpar[k];
        }
        free(order);
        if (L->zpar[n] != L->zpar[0]) return -3; /* cannot happen: n/2 flips, n % 4 == 0 */
    }
    return 0;
}

static void lattice_free(lattice *L)
{
    free(L->six);
    free(L->zpar);
    free(L->alpha);
}

static inline int corner_id(int dx, int dy, int dz) { return dx | (dy << 1) | (dz << 2); }

static inline int det3i(const int a[3], const int b[3], const int c[3])
{
    return a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) +
           a[2] * (b[0] * c[1] - b[1] * c[0]);
}

/* Tets of cube (i,j,k) as local corner ids, positively oriented on the
 * integer template.  Returns the count (5 or 6). */
static int cube_tets(const lattice *L, int i, int j, int k, int tets[6][4])
{
    int nt = 0;
    int five = 0, par5 = 0, cx = 0, cy = 0;
    if (L->split == 1) {
        if (L->six[k]) {
            int a = L->alpha[k];
            int b = (L->zpar[k] + k + a) & 1;
            cx = (i + a) & 1;
            cy = (j + b) & 1;
        } else {
            five = 1;
            par5 = (L->zpar[k] ^ (i + j + k)) & 1; /* local parity of the central tet */
        }
    }
    if (five) {
        int cen[4], m = 0;
        for (int c = 0; c < 8; ++c) {
            int dx = c & 1, dy = (c >> 1) & 1, dz = (c >> 2) & 1;
            if (((dx + dy + dz) & 1) == par5) cen[m++] = c;
        }
        for (int t = 0; t < 4; ++t) tets[nt][t] = cen[t];
        ++nt;
        for (int c = 0; c < 8; ++c) {
            int dx = c & 1, dy = (c >> 1) & 1, dz = (c >> 2) & 1;
            if (((dx + dy + dz) & 1) == par5) continue;
            tets[nt][0] = c;
            tets[nt][1] = corner_id(dx ^ 1, dy, dz);
            tets[nt][2] = corner_id(dx, dy ^ 1, dz);
            tets[nt][3] = corner_id(dx, dy, dz ^ 1);
            ++nt;
        }
    } else {
        static const int PERM[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2},
                                       {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
        for (int p = 0; p < 6; ++p) {
            int v[3] = {cx, cy, 0};
            tets[nt][0] = corner_id(v[0], v[1], v[2]);
            for (int s = 0; s < 3; ++s) {
                v[PERM[p][s]] ^= 1;
                tets[nt][s + 1] = corner_id(v[0], v[1], v[2]);
            }
            ++nt;
        }
    }
    for (int t = 0; t < nt; ++t) { /* orientation from the integer template */
        int o[3][3];
        for (int s = 0; s < 3; ++s) {
            int a = tets[t][0], b = tets[t][s + 1];
            o[s][0] = (b & 1) - (a & 1);
            o[s][1] = ((b >> 1) & 1) - ((a >> 1) & 1);
            o[s][2] = ((b >> 2) & 1) - ((a >> 2) & 1);
        }
        if (det3i(o[0], o[1], o[2]) < 0) {
            int tmp = tets[t][2];
            tets[t][2] = tets[t][3];
            tets[t][3] = tmp;
        }
    }
    return nt;
}

/* 26 lattice offsets, indexed (dx+1) + 3(dy+1) + 9(dz+1); index 13 unused. */
static inline int off_index(int dx, int dy, int dz) { return (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1); }

int mg_sizes(const mg_params *P, int64_t *N, int64_t *E, int64_t *T)
{
    if (P->n < 3 || (P->split != 0 && P->split != 1) || (P->split == 1 && P->n % 4)) return -1;
    int64_t n = P->n, n3 = n * n * n;
    *N = n3;
    if (P->split == 0) {
        *E = 7 * n3;
        *T = 6 * n3;
    } else {
        *E = 6 * n3 + n3 / 2;
        *T = 5 * n3 + n3 / 2;
    }
    return 0;
}

/* Edge id of (a, b), a < b: position of b in a's sorted forward list. */
static inline int64_t edge_of(const int64_t *first, const int32_t *fwd, int64_t a, int64_t b)
{
    for (int64_t e = first[a]; e < first[a + 1]; ++e)
        if (fwd[e] == b) return e;
    return -1;
}

int mg_build(const mg_params *P, int32_t *e2n, double *w, double *vol, double *xyz,
             int32_t *perm, int64_t *stats)
{
    int64_t N, E, T;
    if (mg_sizes(P, &N, &E, &T)) return -1;
    if (!(P->jitter >= 0.0 && P->jitter < 0.5)) return -1;
    lattice L;
    int rc = lattice_init(&L, P);
    if (rc) {
        lattice_free(&L);
        return rc;
    }
    const int n = P->n;
    const double h = 1.0 / n;

    /* positions in generator order */
    double *pos = malloc((size_t)N * 3 * sizeof(double));
    uint32_t *adj = calloc((size_t)N, sizeof(uint32_t));
    int64_t *first = malloc((size_t)(N + 1) * sizeof(int64_t));
    int32_t *fwd = malloc((size_t)E * sizeof(int32_t));
    if (!pos || !adj || !first || !fwd) {
        rc = -2;
        goto out;
    }
    {
        uint64_t s = mg_stream(P->mesh_seed, MG_PURPOSE_JITTER);
        for (int64_t g = 0; g < N; ++g) {
            int64_t i = g % n, j = (g / n) % n, k = g / ((int64_t)n * n);
            int64_t ijk[3] = {i, j, k};
            for (int d = 0; d < 3; ++d) {
                double xi = 2.0 * sm_uniform(&s) - 1.0;
                pos[3 * g + d] = h * (double)ijk[d] + h * P->jitter * xi;
            }
        }
    }

    /* node relabelling: perm[g] = user label of generator node g */
    for (int64_t g = 0; g < N; ++g) perm[g] = (int32_t)g;
    if (P->permute) {
        uint64_t s = mg_stream(P->mesh_seed, MG_PURPOSE_PERM);
        for (int64_t g = N - 1; g > 0; --g) {
            int64_t j = (int64_t)sm_below(&s, (uint64_t)g + 1);
            int32_t t = perm[g];
            perm[g] = perm[j];
            perm[j] = t;
        }
    }

    /* pass 1: adjacency bits from every tet edge */
    int64_t ntets = 0;
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                int tets[6][4];
                int nt = cube_tets(&L, i, j, k, tets);
                ntets += nt;
                for (int t = 0; t < nt; ++t)
                    for (int e = 0; e < 6; ++e) {
                        int cu = tets[t][TET_EDGE[e][0]], cv = tets[t][TET_EDGE[e][1]];
                        int dx = (cv & 1) - (cu & 1), dy = ((cv >> 1) & 1) - ((cu >> 1) & 1),
                            dz = ((cv >> 2) & 1) - ((cu >> 2) & 1);
                        int64_t a = gid(&L, i + (cu & 1), j + ((cu >> 1) & 1), k + ((cu >> 2) & 1));
                        int64_t b = gid(&L, i + (cv & 1), j + ((cv >> 1) & 1), k + ((cv >> 2) & 1));
                        adj[a] |= 1u << off_index(dx, dy, dz);
                        adj[b] |= 1u << off_index(-dx, -dy, -dz);
                    }
            }
    if (ntets != T) {
        rc = -4;
        goto out;
    }

    /* edges: forward neighbours b > a, in lexicographic (a, b) order */
    first[0] = 0;
    for (int64_t a = 0; a < N; ++a) {
        int64_t ai = a % n, aj = (a / n) % n, ak = a / ((int64_t)n * n);
        int64_t nb[27];
        int m = 0;
        for (int o = 0; o < 27; ++o) {
            if (!(adj[a] >> o & 1u)) continue;
            int dx = o % 3 - 1, dy = (o / 3) % 3 - 1, dz = o / 9 - 1;
            int64_t c = gid(&L, ai + dx + n, aj + dy + n, ak + dz + n);
            if (c > a) nb[m++] = c;
        }
        for (int x = 1; x < m; ++x) { /* insertion sort, m <= 26 */
            int64_t v = nb[x];
            int y = x - 1;
            while (y >= 0 && nb[y] > v) {
                nb[y + 1] = nb[y];
                --y;
            }
            nb[y + 1] = v;
        }
        if (first[a] + m > E) {
            rc = -4;
            goto out;
        }
        for (int x = 0; x < m; ++x) {
            fwd[first[a] + x] = (int32_t)nb[x];
            e2n[2 * (first[a] + x)] = perm[a];
            e2n[2 * (first[a] + x) + 1] = perm[nb[x]];
        }
        first[a + 1] = first[a] + m;
    }
    if (first[N] != E) {
        rc = -4;
        goto out;
    }

    /* pass 2: median-dual weights and dual volumes */
    memset(w, 0, (size_t)E * 3 * sizeof(double));
    memset(vol, 0, (size_t)N * sizeof(double));
    int64_t inverted = 0;
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                int tets[6][4];
                int nt = cube_tets(&L, i, j, k, tets);
                for (int t = 0; t < nt; ++t) {
                    double x[12];
                    int64_t g[4];
                    for (int v = 0; v < 4; ++v) {
                        int c = tets[t][v];
                        int ii = i + (c & 1), jj = j + ((c >> 1) & 1), kk = k + ((c >> 2) & 1);
                        g[v] = gid(&L, ii, jj, kk);
                        x[3 * v + 0] = pos[3 * g[v] + 0] + (ii >= n ? 1.0 : 0.0);
                        x[3 * v + 1] = pos[3 * g[v] + 1] + (jj >= n ? 1.0 : 0.0);
                        x[3 * v + 2] = pos[3 * g[v] + 2] + (kk >= n ? 1.0 : 0.0);
                    }
                    double nv[18], vt;
                    mg_tet_dual(x, nv, &vt);
                    if (vt <= 0.0) ++inverted;
                    for (int v = 0; v < 4; ++v) vol[perm[g[v]]] += vt / 4.0;
                    for (int e = 0; e < 6; ++e) {
                        int64_t p = g[TET_EDGE[e][0]], q = g[TET_EDGE[e][1]];
                        int64_t a = p < q ? p : q, b = p < q ? q : p;
                        double sgn = p < q ? 1.0 : -1.0;
                        int64_t id = edge_of(first, fwd, a, b);
                        if (id < 0) {
                            rc = -4;
                            goto out;
                        }
                        for (int d = 0; d < 3; ++d) w[(int64_t)d * E + id] += sgn * nv[3 * e + d];
                    }
                }
            }

    for (int64_t g = 0; g < N; ++g)
        for (int d = 0; d < 3; ++d) xyz[(int64_t)d * N + perm[g]] = pos[3 * g + d];

    if (stats) {
        int64_t n6 = 0;
        if (L.split == 0)
            n6 = N;
        else
            for (int k = 0; k < n; ++k) n6 += L.six[k] ? (int64_t)n * n : 0;
        stats[0] = inverted;
        stats[1] = n6;
        stats[2] = T;
    }
    rc = 0;
out:
    free(pos);
    free(adj);
    free(first);
    free(fwd);
    lattice_free(&L);
    return rc;
}

int mg_tets(const mg_params *P, const int32_t *perm, int32_t *tets_out)
{
    int64_t N, E, T;
    if (mg_sizes(P, &N, &E, &T)) return -1;
    lattice L;
    int rc = lattice_init(&L, P);
    if (rc) {
        lattice_free(&L);
        return rc;
    }
    const int n = P->n;
    int64_t t_out = 0;
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                int tets[6][4];
                int nt = cube_tets(&L, i, j, k, tets);
                for (int t = 0; t < nt; ++t, ++t_out)
                    for (int v = 0; v < 4; ++v) {
                        int c = tets[t][v];
                        int64_t g = gid(&L, i + (c & 1), j + ((c >> 1) & 1), k + ((c >> 2) & 1));
                        tets_out[4 * t_out + v] = perm[g];
                    }
            }
    lattice_free(&L);
    return t_out == T ? 0 : -4;
}

int mg_state(int64_t N, const int32_t *perm, uint64_t seed, double gamma, double *q)
{
    if (N <= 0 || !(gamma > 1.0)) return -1;
    uint64_t s = mg_stream(seed, MG_PURPOSE_STATE);
    for (int64_t g = 0; g < N; ++g) {
        double rho = 0.9 + 0.2 * sm_uniform(&s);
        double u = -0.3 + 0.6 * sm_uniform(&s);
        double v = -0.3 + 0.6 * sm_uniform(&s);
        double w = -0.3 + 0.6 * sm_uniform(&s);
        double p = 0.9 + 0.2 * sm_uniform(&s);
        double phi = sm_uniform(&s);
        int64_t i = perm ? perm[g] : g;
        q[0 * N + i] = rho;
        q[1 * N + i] = rho * u;
        q[2 * N + i] = rho * v;
        q[3 * N + i] = rho * w;
        q[4 * N + i] = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w);
        q[5 * N + i] = rho * phi;
    }
    return 0;
}

/* Edge ids of the six local edges of every tet ((0,1) (0,2) (0,3) (1,2) (1,3)
 * (2,3)), looked up in a CSR of each node's (larger neighbour, edge) pairs
 * built from e2n.  Connectivity only.  Returns 0, or -1 when a tet edge is not
 * in e2n, -7 on allocation failure. */
int mg_tet_edges(int64_t N, int64_t E, const int32_t *e2n, int64_t T, const int32_t *tets,
                 int32_t *out)
{
    static const int LE[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
    int64_t *off = calloc((size_t)N + 1, sizeof(int64_t));
    int32_t *nb = malloc(sizeof(int32_t) * (size_t)(E > 0 ? E : 1));
    int32_t *id = malloc(sizeof(int32_t) * (size_t)(E > 0 ? E : 1));
    int64_t *fill = malloc(sizeof(int64_t) * (size_t)(N > 0 ? N : 1));
    if (!off || !nb || !id || !fill) {
        free(off), free(nb), free(id), free(fill);
        return -7;
    }
    for (int64_t e = 0; e < E; ++e) {
        const int32_t a = e2n[2 * e], b = e2n[2 * e + 1];
        ++off[(a < b ? a : b) + 1];
    }
    for (int64_t i = 0; i < N; ++i) off[i + 1] += off[i];
    for (int64_t i = 0; i < N; ++i) fill[i] = off[i];
    for (int64_t e = 0; e < E; ++e) {
        const int32_t a = e2n[2 * e], b = e2n[2 * e + 1];
        const int32_t lo = a < b ? a : b, hi = a < b ? b : a;
        nb[fill[lo]] = hi;
        id[fill[lo]++] = (int32_t)e;
    }
    int rc = 0;
    for (int64_t t = 0; t < T && !rc; ++t)
        for (int k = 0; k < 6; ++k) {
            const int32_t p = tets[4 * t + LE[k][0]], q = tets[4 * t + LE[k][1]];
            const int32_t lo = p < q ? p : q, hi = p < q ? q : p;
            int32_t found = -1;
            for (int64_t j = off[lo]; j < off[lo + 1]; ++j)
                if (nb[j] == hi) {
                    found = id[j];
                    break;
                }
            if (found < 0) {
                rc = -1;
                break;
            }
            out[6 * t + k] = found;
        }
    free(off), free(nb), free(id), free(fill);
    return rc;
}
