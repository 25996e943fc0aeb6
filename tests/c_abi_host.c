/* A plain C program using the library through include/opflux.h only: a
 * host-only context, a periodic ring of nodes joined to their next two
 * neighbours, a plan, its bit-exact verification, the permutations, and the
 * error paths of a loop without a device.  Prints "ok" and exits 0 on success. */
#include <stdio.h>
#include <stdlib.h>

#include "opflux.h"

#define CHECK(cond, what)                                   \
    do {                                                    \
        if (!(cond)) {                                      \
            fprintf(stderr, "failed: %s\n", what);          \
            return 1;                                       \
        }                                                   \
    } while (0)

int main(void)
{
    enum { N = 4096, E = 2 * N };
    int32_t *e2n = malloc(sizeof(int32_t) * 2 * E);
    int32_t *perm = malloc(sizeof(int32_t) * N);
    int32_t *eperm = malloc(sizeof(int32_t) * E);
    char *seen = calloc(N > E ? N : E, 1);
    CHECK(e2n && perm && eperm && seen, "host allocation");
    for (int i = 0; i < N; ++i) {
        e2n[4 * i + 0] = i;
        e2n[4 * i + 1] = (i + 1) % N;
        e2n[4 * i + 2] = i;
        e2n[4 * i + 3] = (i + 2) % N;
    }
    opf_ctx *ctx = NULL;
    CHECK(opf_init(&ctx, -1) == OPF_OK && ctx, "host-only context");
    opf_set nodes, edges;
    opf_map m;
    CHECK(opf_decl_set(ctx, N, "nodes", &nodes) == OPF_OK, "node set");
    CHECK(opf_decl_set(ctx, E, "edges", &edges) == OPF_OK, "edge set");
    CHECK(opf_decl_map(ctx, edges, nodes, 2, e2n, 0, "e2n", &m) == OPF_OK, "map");
    /* before a plan the internal numbering is the user's */
    CHECK(opf_get_perm(ctx, nodes, perm) == OPF_OK, "permutation before a plan");
    for (int i = 0; i < N; ++i) CHECK(perm[i] == i, "identity before a plan");

    opf_plan_info info;
    CHECK(opf_plan(ctx, m, NULL, &info) == OPF_OK, opf_last_error(ctx));
    CHECK(info.nblocks >= 1 && info.nblock_colours >= 1 && info.owner_ok, "plan statistics");
    opf_plan_report rep;
    CHECK(opf_plan_verify(ctx, m, &rep) == OPF_OK, "plan verification");

    /* the permutations are bijections */
    CHECK(opf_get_perm(ctx, nodes, perm) == OPF_OK, "node permutation");
    for (int i = 0; i < N; ++i) {
        CHECK(perm[i] >= 0 && perm[i] < N && !seen[perm[i]], "node permutation is a bijection");
        seen[perm[i]] = 1;
    }
    for (int i = 0; i < E; ++i) seen[i] = 0;
    CHECK(opf_get_perm(ctx, edges, eperm) == OPF_OK, "edge permutation");
    for (int i = 0; i < E; ++i) {
        CHECK(eperm[i] >= 0 && eperm[i] < E && !seen[eperm[i]], "edge permutation is a bijection");
        seen[eperm[i]] = 1;
    }

    /* without a device, loops refuse to run; bad handles are errors, not crashes */
    opf_dat q, w, res;
    CHECK(opf_decl_dat(ctx, nodes, 6, OPF_F64, NULL, N, "q", &q) == OPF_OK, "dat q");
    CHECK(opf_decl_dat(ctx, edges, 3, OPF_F64, NULL, E, "n", &w) == OPF_OK, "dat n");
    CHECK(opf_decl_dat(ctx, nodes, 6, OPF_F64, NULL, N, "res", &res) == OPF_OK, "dat res");
    CHECK(opf_edge_flux(ctx, edges, m, q, w, res, 1.4, OPF_V_OWNER, OPF_INC, NULL) == OPF_EDEVICE,
          "loop without a device");
    CHECK(opf_edge_flux(ctx, edges, m + 7, q, w, res, 1.4, OPF_V_OWNER, OPF_INC, NULL) ==
              OPF_EINVAL,
          "bad map handle");
    CHECK(opf_finalize(ctx) == OPF_OK, "finalize");
    CHECK(opf_finalize(NULL) == OPF_OK, "finalize(NULL)");
    free(e2n);
    free(perm);
    free(eperm);
    free(seen);
    printf("ok\n");
    return 0;
}
