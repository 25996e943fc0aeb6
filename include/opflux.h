/*
 * opflux.h -- C ABI of the MI355X edge-flux library (libopflux.so).
 *
 * The calls follow the paper's statement of an unstructured-mesh problem
 * (Sec. 2: sets, data on sets, mappings between sets, operations over sets)
 * and the OP2 API built on it (Sec. 3.1): declare sets, an arity-2 map from
 * edges to nodes, data arrays on sets, then run a loop over a set whose
 * arguments say how each array is reached (directly, or through the map) and
 * how it is accessed (READ, WRITE, RW, INC).  As in OP2 (Sec. 3.2), the library
 * owns the maps, may renumber the sets, and decides how a loop is executed;
 * for an indirect loop it builds an execution plan once per map (Sec. 4.1):
 * mini-partitions of consecutive edges, a colouring of the mini-partitions so
 * that partitions of one colour share no node, and a colouring of the edges
 * inside each partition so that edges of one colour share no node.  The same
 * plan also groups the nodes into clusters of consecutive internal labels,
 * each owned by one workgroup that runs every edge touching it and writes its
 * nodes' totals once (the OWNER variant, the owner-compute rule of the paper's
 * distributed back-end applied inside one GPU).
 *
 * Conventions
 *  - Every call returns an int status: OPF_OK (0) or a negative opf_status.
 *    Nothing throws or aborts across the ABI; opf_last_error() gives a message.
 *  - Sizes are int64_t, indices int32_t.  Handles (opf_set, opf_map, opf_dat)
 *    are small non-negative integers valid until opf_finalize().
 *  - A context is not thread-safe.  Loops are asynchronous on the HIP stream
 *    passed as `stream` (a hipStream_t; NULL = the null stream); the library
 *    never synchronises unless asked (opf_sync, opf_plan).
 *  - Streams and library scratch: the direct reductions (RK stage, time
 *    step), the fused edge loop + stage and the gather form of the tet loops
 *    keep partial results in device scratch owned by the context (or by the
 *    plan), shared by every call.  Such a call records an event on its stream;
 *    the next such call on a different stream waits for that event first, so
 *    their uses of the scratch never overlap.  Loops that use no scratch (the
 *    plain edge loops) are not ordered across streams.
 *  - Aliasing: every output (WRITE, RW, INC) must share no byte with any other
 *    argument of the same call, device globals included.  Dats are compared by
 *    the address range their elements cover ([ptr, ptr + ((dim-1)*ld + size)
 *    * elemsize)), so two handles over one buffer are refused (OPF_EINVAL)
 *    before anything is launched.
 *  - Data arrays ("dats") are borrowed device memory in SoA layout: component c
 *    of element k is at ptr[c * ld + k], ld >= set size.  They must be in the
 *    library's internal numbering once a plan has renumbered their set (use
 *    opf_get_perm to move data in and out).  The caller keeps them alive.
 */
#ifndef OPFLUX_H
#define OPFLUX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct opf_ctx opf_ctx;
typedef int32_t opf_set;
typedef int32_t opf_map;
typedef int32_t opf_dat;

/* map value of a direct argument (OP2's OP_ID) */
#define OPF_ID (-1)
/* idx of an argument that reads or increments every column of its map (the
 * tet loops: all four vertices, all six edges). */
#define OPF_ALL (-2)

typedef enum {
    OPF_OK = 0,
    OPF_EINVAL = -1,     /* bad argument value or handle                         */
    OPF_ERANGE = -2,     /* map entry outside the target set                     */
    OPF_ESIZE = -3,      /* set size, dimension or leading dimension mismatch    */
    OPF_ETYPE = -4,      /* data type mismatch                                   */
    OPF_EACCESS = -5,    /* access mode does not match the kernel's signature    */
    OPF_ESTATE = -6,     /* missing or stale plan, wrong call order              */
    OPF_ENOMEM = -7,     /* host or device allocation failed                     */
    OPF_EDEVICE = -8,    /* HIP error, or no device bound to the context         */
    OPF_ENONFINITE = -9, /* a reduction result is not finite                     */
    OPF_EPLAN = -10      /* plan verification found a violation                  */
} opf_status;

typedef enum { OPF_F64 = 0, OPF_F32 = 1 } opf_dtype;

/* access modes of an argument (Sec. 3.1: OP_READ, OP_INC; WRITE and RW for
 * direct arguments and globals; MIN for a global minimum) */
typedef enum { OPF_READ = 0, OPF_WRITE = 1, OPF_RW = 2, OPF_INC = 3, OPF_MIN = 4 } opf_access;

/* The fixed kernel registry (there is no code generation; each kernel has a
 * fixed argument signature, listed at opf_par_loop). */
typedef enum {
    OPF_K_EDGE_FLUX = 0,     /* edge flux, OP_INC of +F / -F into both nodes      */
    OPF_K_EDGE_FLUX_ADJ = 1, /* reverse (adjoint) of the edge flux                */
    OPF_K_RK_STAGE = 2,      /* direct explicit stage update + sum-of-squares     */
    OPF_K_EDGE_SPECRAD = 3,  /* OP_INC of the edge spectral radius into nodes     */
    OPF_K_DT_MIN = 4,        /* direct: global min over nodes of cfl*vol/lambda   */
    OPF_K_LOCAL_DT = 5,      /* direct: per-node step cfl*vol/lambda              */
    OPF_K_EDGE_GRAD = 6,     /* Green-Gauss sums of the state, OP_INC of 18/node  */
    OPF_K_EDGE_FLUX2 = 7,    /* second-order (reconstructed) edge flux, OP_INC    */
    OPF_K_GEOMETRY = 8,      /* tets: median-dual edge weights and node volumes  */
    OPF_K_GEOMETRY_ADJ = 9   /* tets: reverse of GEOMETRY into node coordinates   */
} opf_kernel;

/* How an indirect (edge) loop resolves its increments. */
typedef enum {
    OPF_V_COLOURED = 0, /* mini-partitions staged in LDS, edge colours serialised
                           inside a partition, one launch per partition colour
                           (Sec. 4.1); deterministic                              */
    OPF_V_ATOMIC = 1,   /* one thread per edge, FP64 atomic adds to HBM          */
    OPF_V_OWNER = 2,    /* one workgroup per cluster of consecutive nodes runs
                           every edge touching the cluster (edges between two
                           clusters run twice) and writes its nodes' totals
                           once; single launch, no colours (owner-compute as in
                           Sec. 3.2, at workgroup level).  LDS accumulation uses
                           FP64 LDS atomics, so the summation order varies      */
    OPF_V_COLOURED_LDS_ATOMIC = 3, /* as COLOURED, with LDS atomics in place
                           of the edge colours inside a partition               */
    OPF_V_FLAT = 4      /* one level of colours over the whole edge set (no
                           partitions, no staging): one launch per colour, one
                           thread per edge, plain read-add-write of both ends in
                           HBM -- the single-level counterpart of the Sec. 4.1
                           plan; deterministic.  Unavailable (OPF_EINVAL) when
                           the map needs more than 128 colours                  */
} opf_variant;

typedef enum { OPF_RENUM_NONE = 0, OPF_RENUM_RCM = 1, OPF_RENUM_MORTON = 2 } opf_renumber;

/* ------------------------------------------------------------ context -- */

/* Creates a context bound to HIP device `hip_device`, or a host-only context
 * when hip_device == -1 (declarations, planning and verification work; loops
 * return OPF_EDEVICE).  No device memory is allocated here.
 * Errors: OPF_EINVAL (out == NULL), OPF_EDEVICE (no such device). */
int opf_init(opf_ctx **out, int hip_device);

/* Frees host memory and every device buffer the library allocated (plans,
 * scratch).  Never frees borrowed dats.  Synchronises the device first.
 * Accepts NULL. */
int opf_finalize(opf_ctx *ctx);

/* Message for the last non-zero status returned on ctx ("" if none). The
 * pointer stays valid until the next call on ctx. */
const char *opf_last_error(const opf_ctx *ctx);

/* Optional device allocator for plan arrays and scratch: alloc(user, bytes)
 * returns device memory aligned to at least 16 bytes (the kernels read plan
 * arrays and partial sums as 8- and 16-byte words), or NULL; free(user, ptr)
 * releases it.  Must be set before the first opf_plan.  NULL functions restore
 * hipMalloc / hipFree.
 * Errors: OPF_ESTATE (a plan already exists). */
int opf_set_allocator(opf_ctx *ctx, void *(*alloc_fn)(void *user, size_t bytes),
                      void (*free_fn)(void *user, void *ptr), void *user);

/* ------------------------------------------------------- declarations -- */

/* Declares a set of `size` elements, 0 < size < 2^29 (Sec. 3.1, op_decl_set;
 * the kernels address one component of a dat with 32-bit byte offsets).
 * `name` may be NULL.  Errors: OPF_EINVAL, OPF_ESIZE. */
int opf_decl_set(opf_ctx *ctx, int64_t size, const char *name, opf_set *out);

/* Declares a map from set `from` to set `to` of arity `dim` (Sec. 3.1,
 * op_decl_map; argument order from, to, dim).  `idx` is host memory,
 * row-major from.size x dim; it is COPIED and the library owns the copy.
 * index_base is 0 or 1 (the paper's Fortran maps are 1-based).  Declaring a
 * map again under the same name (same sets, same arity) replaces its entries,
 * keeps its handle and makes its plan stale.
 * Errors: OPF_EINVAL (bad handle, dim < 1, index_base, a name already taken by
 * a map between other sets or of another arity), OPF_ERANGE (an entry outside
 * [0, to.size) after subtracting index_base). */
int opf_decl_map(opf_ctx *ctx, opf_set from, opf_set to, int dim, const int32_t *idx,
                 int index_base, const char *name, opf_map *out);

typedef struct {
    int32_t renumber;      /* opf_renumber                                         */
    int32_t block_size;    /* edges per mini-partition: 64, 128, ..., 2048         */
    int32_t colour_sort;   /* 1: order edges inside each partition by colour       */
    int32_t cluster_size;  /* nodes per owner cluster, 64..4096; 0 = none (the
                              OWNER variant is then unavailable).  Edges are
                              ordered by the cluster pair they join.               */
    int32_t lane_groups;   /* 1: inside each cluster-pair segment, order edges in
                              groups of 64 sharing no node, so the lanes of one
                              wavefront update distinct nodes (OWNER variant)     */
    int32_t owner_compact; /* accepted and ignored: the OWNER variant always
                              reads the edges inside a cluster through 4-byte
                              words of two local offsets                     */
    int32_t bank_spread;   /* 1: place the visits of every 64-lane wavefront of
                              the OWNER variant so that their LDS words fall in
                              distinct banks as far as possible, and choose
                              which end each lane updates first              */
    int32_t halo_order;    /* 1: inside each owner cluster, number the interior
                              nodes first and then the boundary nodes grouped by
                              the other clusters they are joined to, so that a
                              neighbour's gathers of them hit contiguous runs   */
    const double *coords;  /* host, SoA 3 x to.size; required for MORTON          */
} opf_plan_opts;

typedef struct {
    int64_t nblocks;            /* mini-partitions                                */
    int32_t nblock_colours;     /* colours of mini-partitions                     */
    int32_t max_elem_colours;   /* max edge colours inside one partition          */
    double mean_elem_colours;   /* mean edge colours per partition                */
    int64_t sum_unique;         /* sum over partitions of distinct nodes          */
    int32_t max_unique;         /* max distinct nodes of one partition            */
    int32_t min_blocks_per_colour;
    int64_t bandwidth_before;   /* max |i - j| over edges, user numbering         */
    int64_t bandwidth_after;    /* the same after renumbering                     */
    double plan_seconds;        /* host time of opf_plan                          */
    int64_t device_bytes;       /* device memory held by the plan                 */
    int64_t nclusters;          /* owner clusters (0 without clusters)            */
    int64_t owner_edge_visits;  /* edges run by the OWNER variant (>= E)          */
    int32_t max_cluster_segments; /* most cluster-pair segments of one cluster    */
    int32_t owner_ok;           /* 1 when the plan has owner clusters (the OWNER
                                   variant can run)                               */
    int32_t owner_compact;      /* 1 when the plan has owner clusters (the
                                   OWNER kernel then reads interior edges
                                   through 4-byte words of local offsets)         */
    int32_t flat_colours;       /* colours of the flat colouring                  */
    int32_t flat_ok;            /* 1 when the FLAT variant can run (<= 128)       */
    int32_t coloured_ok;        /* 1 when the plan has the two-level colouring;
                                   0 when it could not be built (more than 1024
                                   partition colours, as in an unrenumbered
                                   mesh): the COLOURED variants then refuse to
                                   run (OPF_EINVAL), the others are unaffected   */
} opf_plan_info;

/* Builds the execution plan of an arity-2 map (edges -> nodes) on the host
 * (Sec. 4: renumbering for locality; Sec. 4.1: mini-partitions, two-level
 * colouring; Sec. 4.1.2: colour-sorted edges as an option), verifies it
 * bit-exactly, and uploads it to the device (device contexts only; blocks until
 * the upload is done).  The plan renumbers both sets: afterwards every dat on
 * them must be in internal numbering.  A set can be renumbered by one plan only.
 * Planning the same map again replaces its plan and numbering (move the dats
 * again); the library's device copies of other maps in the old numbering (the
 * tet maps) are dropped and rebuilt on their next use.
 * `opts` NULL means RCM, block_size 512, no colour sort, cluster_size 512,
 * lane groups on, bank spreading on, halo order on.
 * `info` may be NULL.
 * Errors: OPF_EINVAL (dim != 2, self-loop edge, bad options), OPF_ESTATE (a set
 * already renumbered by another plan), OPF_ENOMEM, OPF_EDEVICE, OPF_EPLAN. */
int opf_plan(opf_ctx *ctx, opf_map map, const opf_plan_opts *opts, opf_plan_info *info);

/* Internal label of every user element of set s: new_of_old[user] = internal.
 * Caller-owned host buffer of s.size entries.  Identity if s was not renumbered.
 * For the edge set it gives each user edge's position in internal order. */
int opf_get_perm(const opf_ctx *ctx, opf_set s, int32_t *new_of_old);

/* Read-only view of a plan's host arrays (valid until opf_finalize or the next
 * opf_plan on the same map).  Internal numbering throughout.  Without the
 * two-level colouring (opf_plan_info.coloured_ok == 0) the colouring arrays
 * (block_colour, colour_blocks, colour_offsets, elem_colour, block_ncolours,
 * unique_offsets, unique_nodes, local_idx) are NULL and nblock_colours is 0. */
typedef struct {
    int64_t nnodes, nedges, nblocks;
    int32_t nblock_colours, block_size;
    const int32_t *e2n;            /* [2E] internal map, internal edge order          */
    const int64_t *block_offsets;  /* [nblocks+1] edge range of each partition        */
    const int32_t *block_colour;   /* [nblocks]                                       */
    const int32_t *colour_blocks;  /* [nblocks] partition ids grouped by colour       */
    const int64_t *colour_offsets; /* [nblock_colours+1] into colour_blocks           */
    const uint8_t *elem_colour;    /* [E] edge colour inside its partition            */
    const int32_t *block_ncolours; /* [nblocks] edge colours of each partition        */
    const int64_t *unique_offsets; /* [nblocks+1] into unique_nodes                   */
    const int32_t *unique_nodes;   /* sorted distinct nodes of each partition         */
    const uint16_t *local_idx;     /* [2E] endpoint positions in the partition's list */
    int64_t cluster_size, nclusters;
    const int64_t *cluster_seg_offsets; /* [nclusters+1] into the two arrays below  */
    const int32_t *cluster_seg_start;   /* first edge of each segment of a cluster  */
    const int32_t *cluster_seg_len;     /* edges in the segment                     */
    /* The same work as the OWNER variant reads it: cluster c runs the edges
     * [cluster_range[2c], cluster_range[2c] + cluster_range[2c+1]) -- the edges
     * whose smaller end it owns when they are contiguous, else an empty range --
     * then cluster_list_edges[cluster_list_offsets[c] .. [c+1]), ascending. */
    const int32_t *cluster_range;         /* [2 nclusters]                         */
    const int64_t *cluster_list_offsets;  /* [nclusters+1]                         */
    const int32_t *cluster_list_edges;
    /* Flat colouring: edges flat_edges[flat_offsets[c] .. [c+1]) have colour c
     * (ascending); NULL when the FLAT variant is unavailable. */
    int64_t nflat_colours;
    const int64_t *flat_offsets;  /* [nflat_colours+1]                          */
    const int32_t *flat_edges;    /* [E]                                        */
    const uint8_t *owner_swap;    /* [E] 1: the OWNER kernel updates the edge's
                                     second end first; NULL without bank spreading */
    /* The OWNER kernel's two loops: cluster c first runs the interior block,
     * the first cluster_interior[c] edges of its cluster_range (both ends in
     * c, read through local offsets), then its cut visits
     * cluster_cut_edges[cluster_cut_offsets[c] .. [c+1]), one (edge, owned
     * end) pair each: cluster_cut_ends 0 names the edge's first node, 1 its
     * second.  Every end of every edge is covered exactly once.  The
     * cluster_cutf_* arrays hold the same visits of each cluster in a second
     * order (by foreign node within each run of one other cluster), the one
     * the kernels with wide foreign records use. */
    const int32_t *cluster_interior;     /* [nclusters]                     */
    const int64_t *cluster_cut_offsets;  /* [nclusters+1]                   */
    const int32_t *cluster_cut_edges;
    const uint8_t *cluster_cut_ends;
    const int32_t *cluster_cutf_edges;
    const uint8_t *cluster_cutf_ends;
} opf_plan_view;

int opf_plan_view_get(const opf_ctx *ctx, opf_map map, opf_plan_view *out);

typedef struct {
    int32_t ok;        /* 1 when every property holds                         */
    int32_t property;  /* first violated property 1..9, 0 if none            */
    int64_t where;     /* element (node, edge or partition) of the violation  */
    char message[160];
} opf_plan_report;

/* Host-only, bit-exact verification of a plan: (1) the node relabelling is a
 * bijection; (2) the edge reordering is a bijection and keeps every edge's
 * endpoints and orientation; (3) partitions of one colour share no node; (4)
 * inside a partition, edges of one colour share no node; (5) partitions are
 * contiguous edge ranges of at most block_size edges, grouped by colour;
 * (6) local indices resolve to the map's nodes; (7) colour counts fit their
 * types; (8) every edge is in the work of exactly the owner clusters of its
 * two endpoints, in the segments and in the visit lists alike; (9) every edge
 * has exactly one flat colour and edges of one flat colour share no node.
 * Works without a GPU.  Errors: OPF_EPLAN (report filled),
 * OPF_ESTATE (no plan). */
int opf_plan_verify(const opf_ctx *ctx, opf_map map, opf_plan_report *report);

/* Declares a dat on set s borrowing device memory: dim components of type t,
 * SoA with leading dimension ld >= s.size (Sec. 3.1, op_decl_dat; SoA layout as
 * in Sec. 4.1.2).  Errors: OPF_EINVAL (NULL ptr on a device context, bad
 * handle, dim < 1), OPF_ESIZE (ld < size), OPF_ETYPE (unknown type). */
int opf_decl_dat(opf_ctx *ctx, opf_set s, int dim, int type, void *dev_ptr, int64_t ld,
                 const char *name, opf_dat *out);

/* ------------------------------------------------------------- loops -- */

/* One argument of a loop (Sec. 3.1, op_arg_dat(dat, idx, map, dim, type,
 * access)): idx is the map column (0 or 1) for an indirect argument, or -1
 * with map == OPF_ID for a direct one. */
typedef struct {
    opf_dat dat;
    int32_t idx;
    opf_map map;
    int32_t dim;
    int32_t type;
    int32_t access;
} opf_arg;

/* A global argument: a constant (READ, host or device memory) or a reduction
 * target (INC or MIN, device memory of dim values that the loop updates). */
typedef struct {
    void *ptr;
    int32_t dim;
    int32_t type;
    int32_t access;
    int32_t on_device;
} opf_gbl;

/* Runs kernel k over set s.  Argument signatures (checked; dims are exact):
 *
 *  EDGE_FLUX over edges, any variant:
 *     (q, 0, e2n, 6, T, READ) (q, 1, e2n, 6, T, READ) (n, -1, ID, 3, T, READ)
 *     (res, 0, e2n, 6, F64, INC) (res, 1, e2n, 6, F64, INC)
 *     gbl (gamma, 1, F64, READ, host)
 *   with T = F64, or T = F32 for the FP32-storage form (state, weights and flux
 *   arithmetic in FP32, accumulation into the FP64 residual).  With the OWNER
 *   variant the two node increments may instead be WRITE: res = sum of the
 *   edge contributions, with no need to zero res first (the same holds for the
 *   increments of the other edge kernels).
 *  EDGE_FLUX_ADJ over edges (FP64):
 *     (q,0,e2n,6,READ) (q,1,e2n,6,READ) (n,-1,ID,3,READ)
 *     (rbar,0,e2n,6,READ) (rbar,1,e2n,6,READ)
 *     (qbar,0,e2n,6,INC) (qbar,1,e2n,6,INC) (nbar,-1,ID,3,WRITE)
 *     gbl (gamma, 1, F64, READ, host)
 *  EDGE_SPECRAD over edges: (q,0,e2n,6,T,READ) (q,1,e2n,6,T,READ)
 *     (n,-1,ID,3,T,READ) (lam,0,e2n,1,F64,INC) (lam,1,e2n,1,F64,INC) gbl gamma
 *  EDGE_GRAD over edges (FP64, no globals): (q,0,e2n,6,READ) (q,1,e2n,6,READ)
 *     (n,-1,ID,3,READ) (G,0,e2n,18,INC) (G,1,e2n,18,INC)
 *   Green-Gauss sums over the median-dual cells (the gradient accumulation
 *   loop of Sec. 4's loop tables): +1/2 (q_i + q_j) n_e into G_i and the
 *   negative into G_j; component (v, d) of G is 3v + d; the nodal gradient
 *   is G / vol.
 *  EDGE_FLUX2 over edges (FP64): (q,0,e2n,6,READ) (q,1,e2n,6,READ)
 *     (G,0,e2n,18,READ) (G,1,e2n,18,READ) (vol,0,e2n,1,READ) (vol,1,e2n,1,READ)
 *     (n,-1,ID,3,READ) (dx,-1,ID,3,READ) (res,0,e2n,6,INC) (res,1,e2n,6,INC)
 *     gbl (gamma, 1, F64, READ, host)
 *   the EDGE_FLUX flux of the states reconstructed to the edge midpoint,
 *   q_L = q_i + 1/2 (G_i/vol_i).dx_e and q_R = q_j - 1/2 (G_j/vol_j).dx_e,
 *   dx_e = x_j - x_i; WRITE increments with the OWNER variant as above.
 *  In every edge loop the increment target must not be one of the inputs.
 *  GEOMETRY over tets (variant ATOMIC: one thread per tet scattering with
 *  FP64 atomics, summation order varies; variant OWNER: no atomics, fixed
 *  summation orders, the same bits on every run.  OWNER walks the tets around
 *  each edge, as a chain of vertices, from node coordinates staged per chunk
 *  of nodes (the plan's owner clusters, else 512 nodes) in LDS, writes the
 *  weights and a per-edge volume sum, then sums those per node.  Where a mesh
 *  does not fit that form (a chunk's edges not contiguous in the plan's edge
 *  order, more than 4096 chunk and halo nodes, the tets around an edge not
 *  one fan), each tet's results go to a per-tet buffer that every edge and
 *  node then sums over its incident tets.  The first OWNER call on a pair of
 *  tet maps builds these lists and buffers on the device (about 60 bytes
 *  per edge and 192 per tet; 248 per tet when the forward uses the per-tet
 *  buffer), kept until the maps are declared again or opf_finalize; any
 *  other variant is OPF_EINVAL):
 *     (x, ALL, t2n, 3, F64, READ) (w, ALL, t2e, 3, F64, INC)
 *     (vol, ALL, t2n, 1, F64, INC) gbl (period, 1, F64, READ, host)
 *   With OWNER, w and vol may each be WRITE instead of INC (overwritten).
 *   t2n (tets -> nodes, arity 4) lists positively oriented tets; t2e (tets ->
 *   edges, arity 6) lists their edges in the local order (0,1) (0,2) (0,3)
 *   (1,2) (1,3) (2,3).  The edge set must have been planned (its edge->node
 *   map orients each edge).  Each tet adds the area vectors of its six
 *   median-dual faces, (x_r + x_s - x_p - x_q) x (x_s - x_r) / 24 for local
 *   edge (p, q) with (p, q, r, s) an even permutation of the vertices, to w
 *   (signed from the edge's first to its second node) and a quarter of its
 *   volume to each vertex.  period > 0: vertices are unwrapped to the image
 *   nearest vertex 0 in a periodic box of that side.
 *  GEOMETRY_ADJ over tets (ATOMIC, or OWNER: one thread per tet writes its
 *  four vertex shares to the per-tet buffer, ordered node by node, and each
 *  node sums its run in a fixed order): (x, ALL, t2n, 3, READ)
 *     (wbar, ALL, t2e, 3, READ) (volbar, ALL, t2n, 1, READ)
 *     (xbar, ALL, t2n, 3, INC) gbl period
 *   xbar += (dw/dx)^T wbar + (dvol/dx)^T volbar (shape sensitivities when
 *   wbar is the nbar output of EDGE_FLUX_ADJ).
 *  RK_STAGE over nodes (direct):
 *     (q0,-1,ID,6,T,READ) (res,-1,ID,6,F64,RW) (vol,-1,ID,1,F64,READ)
 *     (q,-1,ID,6,T,WRITE)
 *     gbl (alpha_dt, 1, F64, READ, host) gbl (ss, 6, F64, INC, device)
 *   computes q = q0 - alpha_dt * res / vol in FP64 (rounded once to T), adds
 *   sum_i res_i^2 per component to ss, and zeroes res.  With res READ instead
 *   of RW, res is left untouched (for a following edge loop that WRITEs it).
 *   The sum is deterministic: fixed partition, fixed order.  q must not alias
 *   q0 or res.  Local time stepping: a fifth argument (dt,-1,ID,1,F64,READ)
 *   gives each node its own step; the first global is then the stage
 *   coefficient alpha and q = q0 - alpha * dt_i * res / vol.
 *  LOCAL_DT over nodes (direct): (vol,-1,ID,1,F64,READ) (lam,-1,ID,1,F64,READ)
 *     (dt,-1,ID,1,F64,WRITE) gbl (cfl, 1, F64, READ, host)
 *   dt_i = cfl * vol_i / lam_i with lam the EDGE_SPECRAD sum; dt must not
 *   alias vol or lam.
 *  DT_MIN over nodes (direct): (vol,-1,ID,1,F64,READ) (lam,-1,ID,1,F64,READ)
 *     gbl (cfl, 1, F64, READ, host) gbl (dt, 1, F64, MIN, device)
 *   dt = min(dt, cfl * min_i vol_i / lam_i).
 *
 * Asynchronous on `stream`.  Errors: OPF_EINVAL, OPF_ESIZE, OPF_ETYPE,
 * OPF_EACCESS (signature mismatch), OPF_ESTATE (indirect loop without a
 * current plan), OPF_EDEVICE (host-only context or launch failure). */
int opf_par_loop(opf_ctx *ctx, int kernel, opf_set s, int nargs, const opf_arg *args, int ngbl,
                 const opf_gbl *gbls, int variant, void *stream);

/* Typed wrappers over opf_par_loop with the signatures above.  res_access and
 * qbar_access are OPF_INC, or OPF_WRITE with the OWNER variant; for the stage
 * update res_access is OPF_RW (zero after use) or OPF_READ (keep). */
int opf_edge_flux(opf_ctx *ctx, opf_set edges, opf_map e2n, opf_dat q, opf_dat n, opf_dat res,
                  double gamma, int variant, int res_access, void *stream);
int opf_edge_flux_adjoint(opf_ctx *ctx, opf_set edges, opf_map e2n, opf_dat q, opf_dat n,
                          opf_dat rbar, opf_dat qbar, opf_dat nbar, double gamma, int variant,
                          int qbar_access, void *stream);
int opf_edge_specrad(opf_ctx *ctx, opf_set edges, opf_map e2n, opf_dat q, opf_dat n,
                     opf_dat lam, double gamma, int variant, void *stream);
int opf_edge_gradient(opf_ctx *ctx, opf_set edges, opf_map e2n, opf_dat q, opf_dat n, opf_dat G,
                      int variant, int g_access, void *stream);
int opf_edge_flux2(opf_ctx *ctx, opf_set edges, opf_map e2n, opf_dat q, opf_dat G, opf_dat vol,
                   opf_dat n, opf_dat dx, opf_dat res, double gamma, int variant, int res_access,
                   void *stream);
/* The EDGE_FLUX loop (OWNER variant) and the RK stage update fused: each
 * owner workgroup turns its nodes' residual totals straight into
 * qout = q0 - alpha * res / vol (alpha * dt_i * res / vol when dt >= 0 names a
 * per-node step dat) and adds sum res^2 per component to ss_dev (6 device
 * doubles; per-cluster partials summed in a fixed order).  The residual is not
 * written.  q: node dat (6, T = F64 or F32) read through e2n; n: edge dat
 * (3, T); q0, qout: node dats (6, T); vol: node dat (1, F64).  q may be q0;
 * qout must differ from both (other workgroups still read q).  A fusion of two
 * loops of the paper's iteration (the edge flux and the direct update of
 * Sec. 2), possible because the owner variant completes every node's total
 * inside one workgroup.  Errors: as opf_par_loop; OPF_EINVAL without owner
 * clusters or on aliasing. */
int opf_edge_flux_stage(opf_ctx *ctx, opf_set edges, opf_map e2n, opf_dat q, opf_dat n,
                        opf_dat q0, opf_dat vol, opf_dat dt, opf_dat qout, double gamma,
                        double alpha, double *ss_dev, void *stream);
/* opf_edge_flux_stage for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, checks, kernels and results; the per-cluster
 * partial sums go to a static device array of the library (6 doubles for each
 * of at most 16384 owner clusters, 768 KiB, and 784 bytes for the final sum
 * and its counter; one copy per GPU, resolved by opf_init and held until the
 * process ends) instead of the plan's buffer.  The
 * call allocates nothing (no hipMalloc, no context scratch, no event) and does
 * not order itself against other streams: every call on one GPU, from any
 * context, shares that array, so calls that overlap in time on one GPU race.
 * Every cluster writes its partials before they are summed, and the final
 * sum's counter starts at zero (static initialisation) and returns to zero at
 * the end of every call, so nothing needs clearing between calls.  The plan
 * (opf_plan) must exist already.
 * Errors: as opf_edge_flux_stage; OPF_ESIZE when the plan has more than 16384
 * clusters; OPF_ESTATE when the static array could not be resolved. */
int opf_edge_flux_stage_noalloc(opf_ctx *ctx, opf_set edges, opf_map e2n, opf_dat q, opf_dat n,
                                opf_dat q0, opf_dat vol, opf_dat dt, opf_dat qout, double gamma,
                                double alpha, double *ss_dev, void *stream);
int opf_geometry(opf_ctx *ctx, opf_set tets, opf_map t2n, opf_map t2e, opf_dat x, double period,
                 opf_dat w, opf_dat vol, int variant, void *stream);
int opf_geometry_adjoint(opf_ctx *ctx, opf_set tets, opf_map t2n, opf_map t2e, opf_dat x,
                         double period, opf_dat wbar, opf_dat volbar, opf_dat xbar, int variant,
                         void *stream);
int opf_rk_stage(opf_ctx *ctx, opf_set nodes, opf_dat q0, opf_dat res, opf_dat vol, opf_dat q,
                 double alpha_dt, double *ss_dev, int res_access, void *stream);
int opf_rk_stage_local(opf_ctx *ctx, opf_set nodes, opf_dat q0, opf_dat res, opf_dat vol,
                       opf_dat dt, opf_dat q, double alpha, double *ss_dev, int res_access,
                       void *stream);
int opf_local_dt(opf_ctx *ctx, opf_set nodes, opf_dat vol, opf_dat lam, double cfl, opf_dat dt,
                 void *stream);
int opf_dt_min(opf_ctx *ctx, opf_set nodes, opf_dat vol, opf_dat lam, double cfl,
               double *dt_dev, void *stream);

/* Waits for `stream` and reports asynchronous HIP errors.  Errors: OPF_EDEVICE. */
int opf_sync(opf_ctx *ctx, void *stream);

/* Optional reduction check: reads n doubles from device memory and returns
 * OPF_ENONFINITE if any is NaN or infinite (synchronises `stream`). */
int opf_check_finite(opf_ctx *ctx, const double *dev_ptr, int n, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* OPFLUX_H */
