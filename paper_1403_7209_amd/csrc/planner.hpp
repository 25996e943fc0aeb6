// planner.hpp -- host execution plan of an edge -> node map.
//
// Sec. 4 (renumbering for cache locality, GPS in the paper; RCM or a Morton
// curve here) and Sec. 4.1 (mini-partitions of the execution set, a colouring
// of the partitions so that same-colour partitions share no node, and a
// colouring of the edges inside each partition for one-edge-per-thread
// execution; the plan is built once and reused).  Sec. 4.1.2: optional
// ordering of each partition's edges by colour.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace opf {

constexpr int kMaxBlockColours = 1024;

struct PlanOptions {
    int renumber = 1;  // 0 none, 1 RCM, 2 Morton
    int block_size = 512;
    int colour_sort = 0;
    int cluster_size = 512;          // nodes per owner cluster; 0 = no owner clusters
    int lane_groups = 1;             // reorder each cluster-pair segment into groups of
                                     // 64 edges that share no node
    int bank_spread = 1;             // place the edges of every 64-visit wavefront chunk
                                     // on lanes so their LDS words fall in distinct banks
    int halo_order = 1;              // inside each cluster: interior nodes first, then
                                     // boundary nodes grouped by the clusters they border
    const double *coords = nullptr;  // SoA 3 x N
};

struct Plan {
    int64_t N = 0, E = 0;
    int block_size = 0;
    std::vector<int32_t> node_new;  // [N] internal label of user node
    std::vector<int32_t> edge_new;  // [E] internal position of user edge
    std::vector<int32_t> e2n;       // [2E] internal map in internal edge order
    std::vector<int64_t> block_off; // [nb+1]
    std::vector<int32_t> block_colour;
    std::vector<int32_t> colour_blocks;
    std::vector<int64_t> colour_off;
    std::vector<uint8_t> ecol;       // [E]
    std::vector<int32_t> block_ncol; // [nb]
    std::vector<int64_t> uniq_off;   // [nb+1]
    std::vector<int32_t> uniq;       // sum U_b
    std::vector<uint16_t> lidx;      // [2E]
    // false when the two-level colouring of Sec. 4.1 could not be built (more
    // than kMaxBlockColours partition colours, more than 64 edge colours or
    // 65535 distinct nodes in a partition): the coloured variants are then
    // unavailable and their arrays empty, while the rest of the plan (owner
    // clusters, flat colouring) stays valid
    bool coloured_ok = true;
    std::string coloured_why;
    int32_t nblock_colours = 0;
    int32_t max_elem_colours = 0;
    double mean_elem_colours = 0.0;
    int32_t max_unique = 0;
    int32_t min_blocks_per_colour = 0;
    int64_t bandwidth_before = 0, bandwidth_after = 0;
    double phase_seconds[4] = {0, 0, 0, 0};  // renumber, edge order, partitions, colours
    // Owner clusters: cluster c owns internal nodes [c*K, min((c+1)*K, N)).
    // Edges are ordered so that those joining clusters (x, y), x <= y, form one
    // contiguous segment; cluster c's work is every segment with x == c or
    // y == c, the (c, c) segment first.
    int32_t cluster_size = 0;
    int32_t max_cluster_segments = 0;
    bool owner_ok = false;              // the plan has owner clusters
    std::vector<int64_t> cl_seg_off;    // [ncl+1] into cl_seg_start / cl_seg_len
    std::vector<int32_t> cl_seg_start;  // first internal edge of each segment
    std::vector<int32_t> cl_seg_len;    // edges in the segment
    int64_t owner_edge_visits = 0;      // sum over clusters of their edges
    // The same work as visit lists: cluster c runs the edges
    // [cl_prim[2c], cl_prim[2c] + cl_prim[2c+1]) (the edges whose smaller end
    // it owns, when they are contiguous; else an empty range), then the edges
    // cl_sec_eid[cl_sec_off[c] .. cl_sec_off[c+1]) in ascending order.
    std::vector<int32_t> cl_prim;     // [2 ncl]
    std::vector<int64_t> cl_sec_off;  // [ncl+1]
    std::vector<int32_t> cl_sec_eid;
    // Per internal edge: 1 when the owner kernel should issue the second end's
    // LDS update first (bank spreading); empty when not computed.
    std::vector<uint8_t> owner_swap;
    // The same work as the owner kernel runs it, in two loops.  Cluster c first
    // runs its interior block [cl_prim[2c], cl_prim[2c] + cl_nint[c]): the
    // leading edges of its range with both ends in c, read through local
    // offsets.  Then its cut visits cl_cut_eid[cl_cut_off[c] .. [c+1]): every
    // other (edge, end in c) pair, the end given by cl_cut_end (0: the edge's
    // first node, 1: its second), one owned end per visit, ordered so that the
    // owned ends of 16 consecutive visits fall in distinct LDS banks.  The same
    // visits of each cluster again in cl_cutf_*, ordered within each run (one
    // other cluster) by their foreign node, then their owned node, so that the
    // lanes of a wavefront gather few foreign records: the loops with wide
    // foreign records use this order, the others the bank-spread one.
    std::vector<int32_t> cl_nint;
    std::vector<int64_t> cl_cut_off;
    std::vector<int32_t> cl_cut_eid;
    std::vector<uint8_t> cl_cut_end;
    std::vector<int32_t> cl_cutf_eid;
    std::vector<uint8_t> cl_cutf_end;
    // Flat colouring (one level over all edges; no partitions): edges
    // flat_eid[flat_off[c] .. flat_off[c+1]) have colour c and share no node.
    bool flat_ok = false;  // false when more than 128 colours would be needed
    int32_t flat_colours = 0;
    std::vector<int64_t> flat_off;
    std::vector<int32_t> flat_eid;
    int64_t nclusters() const { return cluster_size ? (N + cluster_size - 1) / cluster_size : 0; }
    int64_t nblocks() const { return block_off.empty() ? 0 : (int64_t)block_off.size() - 1; }
};

// Builds a plan of the map e2n (2E entries, 0-based, user numbering).
// Returns 0, or a negative opf_status with `err` set.
int build_plan(int64_t N, int64_t E, const int32_t *e2n, const PlanOptions &opt, Plan &plan,
               std::string &err);

struct VerifyResult {
    bool ok = true;
    int property = 0;
    int64_t where = -1;
    std::string message;
};

// Bit-exact check of the plan's properties (1..9) against the user map.
VerifyResult verify_plan(const Plan &plan, const int32_t *e2n_user);

}  // namespace opf
