// planner.cpp -- host execution plan of an edge -> node map (see planner.hpp).
#include "planner.hpp"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdlib>
#include <numeric>
#include <thread>

#include "opflux.h"

namespace opf {
namespace {

struct Graph {
    std::vector<int64_t> off;
    std::vector<int32_t> adj;
};

// Symmetric node adjacency; each list ordered by (degree, id) as Cuthill-McKee
// visits neighbours.  A repeated edge gives a repeated neighbour, which the
// traversals below tolerate.
Graph node_graph(int64_t N, int64_t E, const int32_t *e2n)
{
    Graph g;
    g.off.assign(N + 1, 0);
    for (int64_t e = 0; e < E; ++e) {
        ++g.off[e2n[2 * e] + 1];
        ++g.off[e2n[2 * e + 1] + 1];
    }
    for (int64_t i = 0; i < N; ++i) g.off[i + 1] += g.off[i];
    g.adj.resize(g.off[N]);
    std::vector<int64_t> fill(g.off.begin(), g.off.end() - 1);
    for (int64_t e = 0; e < E; ++e) {
        int32_t a = e2n[2 * e], b = e2n[2 * e + 1];
        g.adj[fill[a]++] = b;
        g.adj[fill[b]++] = a;
    }
    for (int64_t i = 0; i < N; ++i) {
        auto b = g.adj.begin() + g.off[i], en = g.adj.begin() + g.off[i + 1];
        std::sort(b, en, [&](int32_t x, int32_t y) {
            int64_t dx = g.off[x + 1] - g.off[x], dy = g.off[y + 1] - g.off[y];
            return dx != dy ? dx < dy : x < y;
        });
    }
    return g;
}

// BFS from r; returns the number of levels and fills `last` with the last level.
int bfs_levels(const Graph &g, int32_t r, std::vector<int32_t> &level, std::vector<int32_t> &queue,
               std::vector<int32_t> &touched, std::vector<int32_t> &last)
{
    for (int32_t t : touched) level[t] = -1;
    touched.clear();
    queue.clear();
    queue.push_back(r);
    level[r] = 0;
    touched.push_back(r);
    int maxl = 0;
    for (size_t h = 0; h < queue.size(); ++h) {
        int32_t v = queue[h];
        for (int64_t k = g.off[v]; k < g.off[v + 1]; ++k) {
            int32_t w = g.adj[k];
            if (level[w] < 0) {
                level[w] = level[v] + 1;
                maxl = std::max(maxl, level[w]);
                queue.push_back(w);
                touched.push_back(w);
            }
        }
    }
    last.clear();
    for (int32_t v : queue)
        if (level[v] == maxl) last.push_back(v);
    return maxl + 1;
}

// Reverse Cuthill-McKee with a pseudo-peripheral start per component
// (George and Liu's iteration: restart from a minimum-degree node of the last
// BFS level while the eccentricity grows).  new_of_old[i] = RCM label.
void rcm(int64_t N, const Graph &g, std::vector<int32_t> &new_of_old)
{
    std::vector<int32_t> level(N, -1), queue, touched, last;
    std::vector<char> done(N, 0);
    std::vector<int32_t> order;
    order.reserve(N);
    queue.reserve(N);
    touched.reserve(N);
    auto deg = [&](int32_t v) { return g.off[v + 1] - g.off[v]; };
    for (int64_t s = 0; s < N; ++s) {
        if (done[s]) continue;
        int32_t r = (int32_t)s;
        int ecc = bfs_levels(g, r, level, queue, touched, last);
        for (int it = 0; it < 16; ++it) {
            int32_t x = last[0];
            for (int32_t v : last)
                if (deg(v) < deg(x) || (deg(v) == deg(x) && v < x)) x = v;
            int e2 = bfs_levels(g, x, level, queue, touched, last);
            if (e2 <= ecc) break;
            ecc = e2;
            r = x;
        }
        size_t head = order.size();
        order.push_back(r);
        done[r] = 1;
        for (size_t h = head; h < order.size(); ++h) {
            int32_t v = order[h];
            for (int64_t k = g.off[v]; k < g.off[v + 1]; ++k) {
                int32_t w = g.adj[k];
                if (!done[w]) {
                    done[w] = 1;
                    order.push_back(w);
                }
            }
        }
    }
    new_of_old.assign(N, 0);
    for (int64_t k = 0; k < N; ++k) new_of_old[order[k]] = (int32_t)(N - 1 - k);
}

inline uint64_t spread3(uint64_t x)  // 21 bits -> every third bit
{
    x &= 0x1fffffULL;
    x = (x | x << 32) & 0x1f00000000ffffULL;
    x = (x | x << 16) & 0x1f0000ff0000ffULL;
    x = (x | x << 8) & 0x100f00f00f00f00fULL;
    x = (x | x << 4) & 0x10c30c30c30c30c3ULL;
    x = (x | x << 2) & 0x1249249249249249ULL;
    return x;
}

void morton(int64_t N, const double *xyz, std::vector<int32_t> &new_of_old)
{
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        lo[d] = hi[d] = xyz[d * N];
        for (int64_t i = 0; i < N; ++i) {
            lo[d] = std::min(lo[d], xyz[d * N + i]);
            hi[d] = std::max(hi[d], xyz[d * N + i]);
        }
    }
    std::vector<uint64_t> key(N);
    for (int64_t i = 0; i < N; ++i) {
        uint64_t k = 0;
        for (int d = 0; d < 3; ++d) {
            double span = hi[d] > lo[d] ? hi[d] - lo[d] : 1.0;
            double t = (xyz[d * N + i] - lo[d]) / span;
            uint64_t c = (uint64_t)std::min(2097151.0, std::max(0.0, t * 2097151.0));
            k |= spread3(c) << d;
        }
        key[i] = k;
    }
    std::vector<int32_t> order(N);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return key[a] < key[b]; });
    new_of_old.assign(N, 0);
    for (int64_t k = 0; k < N; ++k) new_of_old[order[k]] = (int32_t)k;
}

inline int lowest_free(uint64_t used) { return used == ~0ULL ? -1 : __builtin_ctzll(~used); }

// Runs f(0..n-1) on up to 16 host threads (independent iterations only).
template <class F>
void parallel_for(int64_t n, const F &f)
{
    const int64_t nt = std::max<int64_t>(1, std::min<int64_t>({16, (int64_t)std::thread::hardware_concurrency(), n}));
    if (nt <= 1) {
        for (int64_t i = 0; i < n; ++i) f(i);
        return;
    }
    std::atomic<int64_t> next(0);
    std::vector<std::thread> pool;
    for (int64_t t = 0; t < nt; ++t)
        pool.emplace_back([&] {
            for (int64_t i; (i = next.fetch_add(1)) < n;) f(i);
        });
    for (std::thread &th : pool) th.join();
}

// Bank spreading.  The owner kernel's lanes take a cluster's visits in order;
// per lane the LDS words of its owned ends (offset o inside the cluster) are
// updated by two instructions, "first" and "second" end.  The LDS serves a
// quarter-wavefront (16 lanes) per pass and its 8-byte words fall in 16 banks
// (o mod 16), so 16 lanes conflict-free need 16 distinct residues per
// instruction.  quarter_groups() splits a list of visits into groups of 16
// with distinct residues in each slot (first fit over open groups; an edge
// with two owned ends may go either way round), full groups first, so the
// groups line up with quarter-wavefronts.  ends[2t], ends[2t+1]: offsets of
// visit t's ends (-1: not owned); fixed[t] >= 0 forces the orientation.
void quarter_groups(int n, const int32_t *ends, const int8_t *fixed, int lead, std::vector<int> &perm,
                    std::vector<uint8_t> &swap)
{
    struct Group {
        uint16_t a = 0, b = 0;
        std::vector<int> members;
    };
    std::vector<Group> open, done;
    perm.clear();
    swap.assign(n, 0);
    const size_t kMaxOpen = 1024;
    for (int t = 0; t < n; ++t) {
        const int r0 = ends[2 * t] < 0 ? -1 : ends[2 * t] & 15;
        const int r1 = ends[2 * t + 1] < 0 ? -1 : ends[2 * t + 1] & 15;
        int where = -1, orient = 0;
        for (size_t g = 0; g < open.size() && where < 0; ++g)
            for (int o = 0; o < 2; ++o) {
                if (fixed[t] >= 0 && o != fixed[t]) continue;
                const int ra = o ? r1 : r0, rb = o ? r0 : r1;
                if ((ra < 0 || !((open[g].a >> ra) & 1)) && (rb < 0 || !((open[g].b >> rb) & 1))) {
                    where = (int)g;
                    orient = o;
                    break;
                }
            }
        if (where < 0) {
            if (open.size() >= kMaxOpen) {  // too many open groups: close the fullest
                size_t best = 0;
                for (size_t g = 1; g < open.size(); ++g)
                    if (open[g].members.size() > open[best].members.size()) best = g;
                done.push_back(std::move(open[best]));
                open.erase(open.begin() + best);
            }
            open.emplace_back();
            where = (int)open.size() - 1;
            orient = fixed[t] >= 0 ? fixed[t] : 0;
        }
        Group &G = open[where];
        const int ra = orient ? r1 : r0, rb = orient ? r0 : r1;
        if (ra >= 0) G.a |= (uint16_t)(1u << ra);
        if (rb >= 0) G.b |= (uint16_t)(1u << rb);
        G.members.push_back(t);
        swap[t] = (uint8_t)orient;
        if (G.members.size() == 16) {
            done.push_back(std::move(G));
            open.erase(open.begin() + where);
        }
    }
    // full groups line up with quarter-wavefronts; the partial ones go last,
    // except that `lead` visits taken from them fill the quarter that precedes
    // the list (the list starts `lead` lanes before a quarter boundary)
    std::vector<int> full, rest;
    for (const Group &g : done)
        (g.members.size() == 16 ? full : rest).insert(g.members.size() == 16 ? full.end() : rest.end(),
                                                      g.members.begin(), g.members.end());
    for (const Group &g : open) rest.insert(rest.end(), g.members.begin(), g.members.end());
    const int take = std::min<int>(lead, (int)rest.size());
    perm.assign(rest.end() - take, rest.end());
    perm.insert(perm.end(), full.begin(), full.end());
    perm.insert(perm.end(), rest.begin(), rest.end() - take);
}

}  // namespace

int build_plan(int64_t N, int64_t E, const int32_t *e2n_user, const PlanOptions &opt, Plan &P,
               std::string &err)
{
    const int BS = opt.block_size;
    if (BS < 64 || BS > 2048 || (BS & (BS - 1))) {
        err = "block_size must be a power of two in [64, 2048]";
        return OPF_EINVAL;
    }
    const int K = opt.cluster_size;
    if (K != 0 && (K < 64 || K > 4096)) {
        err = "cluster_size must be 0 (no owner clusters) or in [64, 4096]";
        return OPF_EINVAL;
    }
    if (opt.renumber < 0 || opt.renumber > 2) {
        err = "unknown renumbering method";
        return OPF_EINVAL;
    }
    if (opt.renumber == 2 && !opt.coords) {
        err = "Morton renumbering needs node coordinates";
        return OPF_EINVAL;
    }
    if (E < 1 || N < 2) {
        err = "the map needs at least one edge and two nodes";
        return OPF_EINVAL;
    }
    for (int64_t e = 0; e < E; ++e)
        if (e2n_user[2 * e] == e2n_user[2 * e + 1]) {
            err = "edge " + std::to_string(e) + " joins a node to itself";
            return OPF_EINVAL;
        }
    P = Plan();
    P.N = N;
    P.E = E;
    P.block_size = BS;
    P.cluster_size = K;

    auto t0 = std::chrono::steady_clock::now();
    auto lap = [&](int k) {
        auto t1 = std::chrono::steady_clock::now();
        P.phase_seconds[k] = std::chrono::duration<double>(t1 - t0).count();
        t0 = t1;
    };
    // (1) node renumbering
    if (opt.renumber == 1) {
        Graph g = node_graph(N, E, e2n_user);
        rcm(N, g, P.node_new);
    } else if (opt.renumber == 2) {
        morton(N, opt.coords, P.node_new);
    } else {
        P.node_new.resize(N);
        std::iota(P.node_new.begin(), P.node_new.end(), 0);
    }

    // (1b) inside each owner cluster, interior nodes first, then the nodes on
    // the cluster's boundary grouped by the other clusters they are joined to:
    // a neighbouring cluster then gathers its halo from a few contiguous runs
    // of each state component instead of scattered words
    if (K > 0 && opt.halo_order) {
        std::vector<int32_t> fmin(N, INT32_MAX), fmax(N, -1);
        for (int64_t e = 0; e < E; ++e) {
            const int32_t a = P.node_new[e2n_user[2 * e]], b = P.node_new[e2n_user[2 * e + 1]];
            const int32_t ca = a / K, cb = b / K;
            if (ca == cb) continue;
            fmin[a] = std::min(fmin[a], cb);
            fmax[a] = std::max(fmax[a], cb);
            fmin[b] = std::min(fmin[b], ca);
            fmax[b] = std::max(fmax[b], ca);
        }
        std::vector<int32_t> relabel(N);
        const int64_t ncl = (N + K - 1) / K;
        parallel_for(ncl, [&](int64_t c) {
            const int32_t lo = (int32_t)(c * K), hi = (int32_t)std::min<int64_t>(N, (c + 1) * K);
            std::vector<int32_t> v(hi - lo);
            std::iota(v.begin(), v.end(), lo);
            std::stable_sort(v.begin(), v.end(), [&](int32_t x, int32_t y) {
                if ((fmax[x] >= 0) != (fmax[y] >= 0)) return fmax[x] < 0;
                if (fmin[x] != fmin[y]) return fmin[x] < fmin[y];
                return fmax[x] < fmax[y];
            });
            for (int32_t k = 0; k < hi - lo; ++k) relabel[v[k]] = lo + k;
        });
        for (int64_t i = 0; i < N; ++i) P.node_new[i] = relabel[P.node_new[i]];
    }

    lap(0);
    // (2) relabel and order edges by (min, max) internal node: counting sort by
    // the smaller endpoint, then by the larger one inside each bucket.
    std::vector<int64_t> cnt(N + 1, 0);
    for (int64_t e = 0; e < E; ++e) {
        int32_t a = P.node_new[e2n_user[2 * e]], b = P.node_new[e2n_user[2 * e + 1]];
        ++cnt[std::min(a, b) + 1];
        P.bandwidth_before = std::max<int64_t>(
            P.bandwidth_before, std::llabs((int64_t)e2n_user[2 * e] - e2n_user[2 * e + 1]));
        P.bandwidth_after = std::max<int64_t>(P.bandwidth_after, std::llabs((int64_t)a - b));
    }
    for (int64_t i = 0; i < N; ++i) cnt[i + 1] += cnt[i];
    std::vector<int32_t> order(E);  // order[k] = user edge at internal position k
    {
        std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
        for (int64_t e = 0; e < E; ++e) {
            int32_t a = P.node_new[e2n_user[2 * e]], b = P.node_new[e2n_user[2 * e + 1]];
            order[fill[std::min(a, b)]++] = (int32_t)e;
        }
        auto hi = [&](int32_t e) {
            return std::max(P.node_new[e2n_user[2 * e]], P.node_new[e2n_user[2 * e + 1]]);
        };
        for (int64_t i = 0; i < N; ++i)
            std::sort(order.begin() + cnt[i], order.begin() + cnt[i + 1],
                      [&](int32_t x, int32_t y) { return hi(x) != hi(y) ? hi(x) < hi(y) : x < y; });
        // group the edges of each cluster of smaller endpoints by the cluster of
        // their larger endpoint: one contiguous segment per cluster pair
        for (int64_t c0 = 0; K > 0 && c0 < N; c0 += K) {
            const int64_t c1 = std::min<int64_t>(c0 + K, N);
            std::stable_sort(order.begin() + cnt[c0], order.begin() + cnt[c1],
                             [&](int32_t x, int32_t y) { return hi(x) / K < hi(y) / K; });
        }
    }
    P.e2n.resize(2 * E);
    for (int64_t k = 0; k < E; ++k) {
        P.e2n[2 * k] = P.node_new[e2n_user[2 * order[k]]];
        P.e2n[2 * k + 1] = P.node_new[e2n_user[2 * order[k] + 1]];
    }

    lap(1);
    // (2b) inside each cluster-pair segment, order edges into groups of 64 that
    // share no node (first fit over up to 64 x 64 open groups), so that the 64
    // lanes of a wavefront running 64 consecutive edges update 128 distinct nodes
    if (K > 0 && opt.lane_groups) {
        std::vector<uint64_t> mask(N, 0);  // per node: groups of the current window
        std::vector<int32_t> touched, grp_of, ord;
        std::vector<int32_t> gsize;
        int64_t k = 0;
        while (k < E) {
            auto key = [&](int64_t t) {
                const int32_t a = P.node_new[e2n_user[2 * order[t]]], b = P.node_new[e2n_user[2 * order[t] + 1]];
                return std::make_pair(std::min(a, b) / K, std::max(a, b) / K);
            };
            const auto kk = key(k);
            int64_t k1 = k + 1;
            while (k1 < E && key(k1) == kk) ++k1;
            const int64_t n = k1 - k;
            if (n > 64) {
                grp_of.assign(n, -1);
                int base = 0;  // first group of the current window of 64 groups
                int64_t left = n;
                while (left > 0) {
                    gsize.assign(64, 0);
                    uint64_t full = 0;
                    for (int32_t v : touched) mask[v] = 0;
                    touched.clear();
                    for (int64_t t = 0; t < n && full != ~0ULL; ++t) {
                        if (grp_of[t] >= 0) continue;
                        const int32_t a = P.node_new[e2n_user[2 * order[k + t]]];
                        const int32_t b = P.node_new[e2n_user[2 * order[k + t] + 1]];
                        const uint64_t busy = mask[a] | mask[b] | full;
                        if (busy == ~0ULL) continue;
                        const int g = __builtin_ctzll(~busy);
                        if (!mask[a]) touched.push_back(a);
                        if (!mask[b]) touched.push_back(b);
                        mask[a] |= 1ULL << g;
                        mask[b] |= 1ULL << g;
                        if (++gsize[g] == 64) full |= 1ULL << g;
                        grp_of[t] = base + g;
                        --left;
                    }
                    base += 64;
                }
                for (int32_t v : touched) mask[v] = 0;
                touched.clear();
                ord.resize(n);
                std::iota(ord.begin(), ord.end(), 0);
                std::stable_sort(ord.begin(), ord.end(),
                                 [&](int32_t x, int32_t y) { return grp_of[x] < grp_of[y]; });
                std::vector<int32_t> tmp(order.begin() + k, order.begin() + k1);
                for (int64_t t = 0; t < n; ++t) order[k + t] = tmp[ord[t]];
            }
            k = k1;
        }
        for (int64_t t = 0; t < E; ++t) {
            P.e2n[2 * t] = P.node_new[e2n_user[2 * order[t]]];
            P.e2n[2 * t + 1] = P.node_new[e2n_user[2 * order[t] + 1]];
        }
    }

    // (2c) bank spreading of the owner kernel's wavefront chunks over each
    // cluster's range of edges (edges whose smaller end it owns); the ranges are
    // independent, so they are spread by a few host threads
    std::vector<uint8_t> swap_user;
    if (K > 0 && opt.bank_spread) {
        swap_user.assign(E, 0);
        std::vector<std::pair<int64_t, int64_t>> ranges;
        for (int64_t k = 0; k < E;) {
            const int64_t c = std::min(P.e2n[2 * k], P.e2n[2 * k + 1]) / K;
            int64_t k1 = k + 1;
            while (k1 < E && std::min(P.e2n[2 * k1], P.e2n[2 * k1 + 1]) / K == c) ++k1;
            ranges.emplace_back(k, k1);
            k = k1;
        }
        parallel_for((int64_t)ranges.size(), [&](int64_t r) {
            const int64_t k = ranges[r].first, k1 = ranges[r].second;
            const int64_t c = std::min(P.e2n[2 * k], P.e2n[2 * k + 1]) / K, v0 = c * K;
            std::vector<int32_t> ends, tmp_order, tmp_e2n;
            std::vector<int8_t> fixed;
            std::vector<int> perm;
            std::vector<uint8_t> sw;
            // one segment (edges to one neighbour cluster, or inside the
            // cluster) at a time, so that a wavefront's lanes gather from one
            // place and take the same branch
            for (int64_t s0 = k; s0 < k1;) {
                const int64_t cx = std::max(P.e2n[2 * s0], P.e2n[2 * s0 + 1]) / K;
                int64_t s1 = s0 + 1;
                while (s1 < k1 && std::max(P.e2n[2 * s1], P.e2n[2 * s1 + 1]) / K == cx) ++s1;
                const int64_t n = s1 - s0;
                ends.assign(2 * n, -1);
                fixed.assign(n, -1);
                tmp_order.assign(order.begin() + s0, order.begin() + s1);
                tmp_e2n.assign(P.e2n.begin() + 2 * s0, P.e2n.begin() + 2 * s1);
                for (int64_t t = 0; t < n; ++t)
                    for (int h = 0; h < 2; ++h) {
                        const int64_t v = tmp_e2n[2 * t + h];
                        if (v / K == c) ends[2 * t + h] = (int32_t)(v - v0);
                    }
                const int lead = (int)((16 - (s0 - k) % 16) % 16);
                quarter_groups((int)n, ends.data(), fixed.data(), lead, perm, sw);
                for (int64_t t = 0; t < n; ++t) {
                    order[s0 + t] = tmp_order[perm[t]];
                    P.e2n[2 * (s0 + t)] = tmp_e2n[2 * perm[t]];
                    P.e2n[2 * (s0 + t) + 1] = tmp_e2n[2 * perm[t] + 1];
                    swap_user[order[s0 + t]] = sw[perm[t]];
                }
                s0 = s1;
            }
        });
    }

    // (3) mini-partitions of consecutive edges
    const int64_t nb = (E + BS - 1) / BS;
    P.block_off.resize(nb + 1);
    for (int64_t b = 0; b <= nb; ++b) P.block_off[b] = std::min<int64_t>(b * BS, E);

    // (5) edge colours inside each partition; (6) distinct nodes and local indices
    P.ecol.assign(E, 0);
    P.block_ncol.assign(nb, 0);
    P.lidx.resize(2 * E);
    P.uniq_off.assign(nb + 1, 0);
    P.uniq.reserve((size_t)(E / 2));
    std::vector<int32_t> loc(N, -1);
    std::vector<uint64_t> lmask;
    std::vector<int32_t> nodes;
    int64_t ncol_sum = 0;
    for (int64_t b = 0; b < nb; ++b) {
        const int64_t e0 = P.block_off[b], e1 = P.block_off[b + 1];
        nodes.clear();
        for (int64_t k = e0; k < e1; ++k) {
            nodes.push_back(P.e2n[2 * k]);
            nodes.push_back(P.e2n[2 * k + 1]);
        }
        std::sort(nodes.begin(), nodes.end());
        nodes.erase(std::unique(nodes.begin(), nodes.end()), nodes.end());
        for (size_t u = 0; u < nodes.size(); ++u) loc[nodes[u]] = (int32_t)u;
        lmask.assign(nodes.size(), 0);
        int ncol = 0;
        for (int64_t k = e0; k < e1; ++k) {
            int32_t li = loc[P.e2n[2 * k]], lj = loc[P.e2n[2 * k + 1]];
            P.lidx[2 * k] = (uint16_t)li;
            P.lidx[2 * k + 1] = (uint16_t)lj;
            int c = lowest_free(lmask[li] | lmask[lj]);
            if (c < 0 || c > 255) {
                P.coloured_ok = false;
                P.coloured_why = "more than 64 edge colours in partition " + std::to_string(b);
                break;
            }
            lmask[li] |= 1ULL << c;
            lmask[lj] |= 1ULL << c;
            P.ecol[k] = (uint8_t)c;
            ncol = std::max(ncol, c + 1);
        }
        for (int32_t v : nodes) loc[v] = -1;
        P.block_ncol[b] = ncol;
        ncol_sum += ncol;
        P.max_elem_colours = std::max(P.max_elem_colours, ncol);
        P.uniq.insert(P.uniq.end(), nodes.begin(), nodes.end());
        P.uniq_off[b + 1] = (int64_t)P.uniq.size();
        P.max_unique = std::max<int32_t>(P.max_unique, (int32_t)nodes.size());
        if (nodes.size() > 65535 && P.coloured_ok) {
            P.coloured_ok = false;
            P.coloured_why = "partition with more than 65535 distinct nodes";
        }
        if (!P.coloured_ok) break;
    }
    P.mean_elem_colours = (double)ncol_sum / (double)nb;

    // (7) optional: order each partition's edges by colour (stable)
    if (opt.colour_sort && P.coloured_ok) {
        std::vector<int32_t> idx;
        std::vector<int32_t> t_e2n, t_order;
        std::vector<uint16_t> t_lidx;
        std::vector<uint8_t> t_col;
        for (int64_t b = 0; b < nb; ++b) {
            const int64_t e0 = P.block_off[b], n = P.block_off[b + 1] - e0;
            idx.resize(n);
            std::iota(idx.begin(), idx.end(), 0);
            std::stable_sort(idx.begin(), idx.end(),
                             [&](int32_t x, int32_t y) { return P.ecol[e0 + x] < P.ecol[e0 + y]; });
            t_e2n.assign(P.e2n.begin() + 2 * e0, P.e2n.begin() + 2 * (e0 + n));
            t_lidx.assign(P.lidx.begin() + 2 * e0, P.lidx.begin() + 2 * (e0 + n));
            t_col.assign(P.ecol.begin() + e0, P.ecol.begin() + e0 + n);
            t_order.assign(order.begin() + e0, order.begin() + e0 + n);
            for (int64_t k = 0; k < n; ++k) {
                int32_t s = idx[k];
                P.e2n[2 * (e0 + k)] = t_e2n[2 * s];
                P.e2n[2 * (e0 + k) + 1] = t_e2n[2 * s + 1];
                P.lidx[2 * (e0 + k)] = t_lidx[2 * s];
                P.lidx[2 * (e0 + k) + 1] = t_lidx[2 * s + 1];
                P.ecol[e0 + k] = t_col[s];
                order[e0 + k] = t_order[s];
            }
        }
    }
    P.edge_new.resize(E);
    for (int64_t k = 0; k < E; ++k) P.edge_new[order[k]] = (int32_t)k;
    if (!swap_user.empty()) {
        P.owner_swap.resize(E);
        for (int64_t k = 0; k < E; ++k) P.owner_swap[k] = swap_user[order[k]];
    }

    // owner clusters: segments of constant (cluster(min), cluster(max)); a
    // partition may have reordered edges by colour, so segments are formed on
    // the final order and a pair may yield more than one segment
    if (K > 0) {
        const int64_t ncl = P.nclusters();
        std::vector<std::vector<std::pair<int32_t, int32_t>>> segs(ncl);
        int64_t k = 0;
        while (k < E) {
            const int32_t a = std::min(P.e2n[2 * k], P.e2n[2 * k + 1]) / K;
            const int32_t b = std::max(P.e2n[2 * k], P.e2n[2 * k + 1]) / K;
            int64_t k1 = k + 1;
            while (k1 < E && std::min(P.e2n[2 * k1], P.e2n[2 * k1 + 1]) / K == a &&
                   std::max(P.e2n[2 * k1], P.e2n[2 * k1 + 1]) / K == b)
                ++k1;
            const std::pair<int32_t, int32_t> sg((int32_t)k, (int32_t)(k1 - k));
            if (a == b)
                segs[a].insert(segs[a].begin(), sg);
            else {
                segs[a].push_back(sg);
                segs[b].push_back(sg);
            }
            k = k1;
        }
        P.cl_seg_off.assign(ncl + 1, 0);
        P.max_cluster_segments = 0;
        for (int64_t c = 0; c < ncl; ++c) {
            P.cl_seg_off[c + 1] = P.cl_seg_off[c] + (int64_t)segs[c].size();
            P.max_cluster_segments = std::max<int32_t>(P.max_cluster_segments, (int32_t)segs[c].size());
        }
        P.cl_seg_start.resize(P.cl_seg_off[ncl]);
        P.cl_seg_len.resize(P.cl_seg_off[ncl]);
        P.owner_edge_visits = 0;
        for (int64_t c = 0; c < ncl; ++c)
            for (size_t s = 0; s < segs[c].size(); ++s) {
                P.cl_seg_start[P.cl_seg_off[c] + s] = segs[c][s].first;
                P.cl_seg_len[P.cl_seg_off[c] + s] = segs[c][s].second;
                P.owner_edge_visits += segs[c][s].second;
            }
        // visit lists: the contiguous range of edges whose smaller end lies in
        // the cluster, then every other edge that touches it
        std::vector<int64_t> first(ncl, -1), last(ncl, -1), cnt(ncl, 0);
        for (int64_t e = 0; e < E; ++e) {
            const int64_t a = std::min(P.e2n[2 * e], P.e2n[2 * e + 1]) / K;
            if (first[a] < 0) first[a] = e;
            last[a] = e;
            ++cnt[a];
        }
        P.cl_prim.assign(2 * ncl, 0);
        for (int64_t c = 0; c < ncl; ++c)
            if (cnt[c] > 0 && last[c] - first[c] + 1 == cnt[c]) {
                P.cl_prim[2 * c] = (int32_t)first[c];
                P.cl_prim[2 * c + 1] = (int32_t)cnt[c];
            }
        auto in_prim = [&](int64_t c, int64_t e) {
            return e >= P.cl_prim[2 * c] && e < (int64_t)P.cl_prim[2 * c] + P.cl_prim[2 * c + 1];
        };
        P.cl_sec_off.assign(ncl + 1, 0);
        for (int pass = 0; pass < 2; ++pass) {
            std::vector<int64_t> fill(P.cl_sec_off.begin(), P.cl_sec_off.end() - 1);
            for (int64_t e = 0; e < E; ++e) {
                const int64_t a = P.e2n[2 * e] / K, b = P.e2n[2 * e + 1] / K;
                const int64_t cs[2] = {a, b};
                for (int t = 0; t < (a == b ? 1 : 2); ++t) {
                    if (in_prim(cs[t], e)) continue;
                    if (pass == 0)
                        ++P.cl_sec_off[cs[t] + 1];
                    else
                        P.cl_sec_eid[fill[cs[t]]++] = (int32_t)e;
                }
            }
            if (pass == 0) {
                for (int64_t c = 0; c < ncl; ++c) P.cl_sec_off[c + 1] += P.cl_sec_off[c];
                P.cl_sec_eid.resize(P.cl_sec_off[ncl]);
            }
        }
        // bank spreading of the listed visits: chunks follow the kernel's
        // positions, which continue after the cluster's edge range
        if (opt.bank_spread && !P.owner_swap.empty()) {
            // the listed visits have one owned end each, whose instruction the
            // edge's flag (set for the cluster of its smaller end) already fixes
            parallel_for(ncl, [&](int64_t c) {
                const int64_t s0 = P.cl_sec_off[c], ns = P.cl_sec_off[c + 1] - s0;
                std::vector<int32_t> ends, tmp;
                std::vector<int8_t> fixed;
                std::vector<int> perm;
                std::vector<uint8_t> sw;
                // one neighbour cluster at a time (the list is in edge order,
                // which groups the edges by the cluster of their smaller end)
                for (int64_t a = 0; a < ns;) {
                    const int64_t ea = P.cl_sec_eid[s0 + a];
                    const int64_t cx = std::min(P.e2n[2 * ea], P.e2n[2 * ea + 1]) / K;
                    int64_t b = a + 1;
                    while (b < ns) {
                        const int64_t eb = P.cl_sec_eid[s0 + b];
                        if (std::min(P.e2n[2 * eb], P.e2n[2 * eb + 1]) / K != cx) break;
                        ++b;
                    }
                    const int64_t n = b - a;
                    ends.assign(2 * n, -1);
                    fixed.assign(n, 0);
                    tmp.assign(P.cl_sec_eid.begin() + s0 + a, P.cl_sec_eid.begin() + s0 + b);
                    for (int64_t t = 0; t < n; ++t) {
                        const int64_t e = tmp[t];
                        for (int h = 0; h < 2; ++h) {
                            const int64_t v = P.e2n[2 * e + h];
                            if (v / K == c) ends[2 * t + h] = (int32_t)(v - c * K);
                        }
                        fixed[t] = (int8_t)P.owner_swap[e];
                    }
                    const int64_t pos = P.cl_prim[2 * c + 1] + a;  // kernel position of the run
                    const int lead = (int)((16 - pos % 16) % 16);
                    quarter_groups((int)n, ends.data(), fixed.data(), lead, perm, sw);
                    for (int64_t t = 0; t < n; ++t) P.cl_sec_eid[s0 + a + t] = tmp[perm[t]];
                    a = b;
                }
            });
        }
        // the owner kernel's two loops: the interior block of each cluster
        // (leading edges of its range with both ends in it), then its cut
        // visits, one (edge, owned end) pair each: the rest of its range, then
        // its listed edges, one neighbour cluster at a time, each run spread
        // over LDS banks by its owned ends
        P.cl_nint.assign(ncl, 0);
        for (int64_t c = 0; c < ncl; ++c) {
            const int64_t p0 = P.cl_prim[2 * c], pn = P.cl_prim[2 * c + 1];
            int64_t t = 0;
            while (t < pn && P.e2n[2 * (p0 + t)] / K == c && P.e2n[2 * (p0 + t) + 1] / K == c) ++t;
            P.cl_nint[c] = (int32_t)t;
        }
        std::vector<std::vector<int32_t>> cut_eid(ncl), cutf_eid(ncl);
        std::vector<std::vector<uint8_t>> cut_end(ncl), cutf_end(ncl);
        parallel_for(ncl, [&](int64_t c) {
            std::vector<int64_t> src;
            const int64_t p0 = P.cl_prim[2 * c], pn = P.cl_prim[2 * c + 1];
            for (int64_t e = p0 + P.cl_nint[c]; e < p0 + pn; ++e) src.push_back(e);
            for (int64_t s = P.cl_sec_off[c]; s < P.cl_sec_off[c + 1]; ++s) src.push_back(P.cl_sec_eid[s]);
            std::vector<int32_t> &ve = cut_eid[c];
            std::vector<uint8_t> &vh = cut_end[c];
            for (int64_t e : src)
                for (int h = 0; h < 2; ++h)
                    if (P.e2n[2 * e + h] / K == c) {
                        ve.push_back((int32_t)e);
                        vh.push_back((uint8_t)h);
                    }
            {
                // the second order: each run sorted by (foreign node, owned node)
                const int64_t n = (int64_t)ve.size();
                auto foreign = [&](int64_t t) { return P.e2n[2 * ve[t] + (1 - vh[t])]; };
                auto owned = [&](int64_t t) { return P.e2n[2 * ve[t] + vh[t]]; };
                std::vector<int64_t> idx(n);
                std::iota(idx.begin(), idx.end(), 0);
                for (int64_t a = 0; a < n;) {
                    int64_t b = a + 1;
                    while (b < n && foreign(b) / K == foreign(a) / K) ++b;
                    std::stable_sort(idx.begin() + a, idx.begin() + b, [&](int64_t x, int64_t y) {
                        if (foreign(x) != foreign(y)) return foreign(x) < foreign(y);
                        return owned(x) < owned(y);
                    });
                    a = b;
                }
                cutf_eid[c].resize(n);
                cutf_end[c].resize(n);
                for (int64_t t = 0; t < n; ++t) {
                    cutf_eid[c][t] = ve[idx[t]];
                    cutf_end[c][t] = vh[idx[t]];
                }
            }
            if (!opt.bank_spread) return;
            std::vector<int32_t> ends, te;
            std::vector<uint8_t> th;
            std::vector<int8_t> fixed;
            std::vector<int> perm;
            std::vector<uint8_t> sw;
            const int64_t n = (int64_t)ve.size();
            for (int64_t a = 0; a < n;) {
                auto other = [&](int64_t t) { return P.e2n[2 * ve[t] + (1 - vh[t])] / K; };
                int64_t b = a + 1;
                while (b < n && other(b) == other(a)) ++b;
                const int64_t m = b - a;
                ends.assign(2 * m, -1);
                fixed.assign(m, 0);
                for (int64_t t = 0; t < m; ++t)
                    ends[2 * t] = (int32_t)(P.e2n[2 * ve[a + t] + vh[a + t]] - c * K);
                const int lead = (int)((16 - a % 16) % 16);
                quarter_groups((int)m, ends.data(), fixed.data(), lead, perm, sw);
                te.assign(ve.begin() + a, ve.begin() + b);
                th.assign(vh.begin() + a, vh.begin() + b);
                for (int64_t t = 0; t < m; ++t) {
                    ve[a + t] = te[perm[t]];
                    vh[a + t] = th[perm[t]];
                }
                a = b;
            }
        });
        P.cl_cut_off.assign(ncl + 1, 0);
        for (int64_t c = 0; c < ncl; ++c) P.cl_cut_off[c + 1] = P.cl_cut_off[c] + (int64_t)cut_eid[c].size();
        P.cl_cut_eid.resize(P.cl_cut_off[ncl]);
        P.cl_cut_end.resize(P.cl_cut_off[ncl]);
        P.cl_cutf_eid.resize(P.cl_cut_off[ncl]);
        P.cl_cutf_end.resize(P.cl_cut_off[ncl]);
        for (int64_t c = 0; c < ncl; ++c) {
            std::copy(cut_eid[c].begin(), cut_eid[c].end(), P.cl_cut_eid.begin() + P.cl_cut_off[c]);
            std::copy(cut_end[c].begin(), cut_end[c].end(), P.cl_cut_end.begin() + P.cl_cut_off[c]);
            std::copy(cutf_eid[c].begin(), cutf_eid[c].end(), P.cl_cutf_eid.begin() + P.cl_cut_off[c]);
            std::copy(cutf_end[c].begin(), cutf_end[c].end(), P.cl_cutf_end.begin() + P.cl_cut_off[c]);
        }
        P.owner_ok = true;
    }

    // flat colouring: one level over the whole edge set, each edge in edge order
    // takes the lowest colour free at both of its ends (at most 128 colours)
    {
        std::vector<uint64_t> used(2 * (size_t)N, 0);
        std::vector<uint8_t> col(E);
        int ncol = 0;
        P.flat_ok = true;
        for (int64_t e = 0; e < E && P.flat_ok; ++e) {
            const int64_t a = P.e2n[2 * e], b = P.e2n[2 * e + 1];
            int c = lowest_free(used[2 * a] | used[2 * b]);
            if (c < 0) {
                const int c1 = lowest_free(used[2 * a + 1] | used[2 * b + 1]);
                c = c1 < 0 ? -1 : 64 + c1;
            }
            if (c < 0) {
                P.flat_ok = false;
                break;
            }
            const uint64_t bit = 1ULL << (c & 63);
            used[2 * a + (c >> 6)] |= bit;
            used[2 * b + (c >> 6)] |= bit;
            col[e] = (uint8_t)c;
            ncol = std::max(ncol, c + 1);
        }
        if (P.flat_ok) {
            P.flat_colours = ncol;
            P.flat_off.assign(ncol + 1, 0);
            for (int64_t e = 0; e < E; ++e) ++P.flat_off[col[e] + 1];
            for (int c = 0; c < ncol; ++c) P.flat_off[c + 1] += P.flat_off[c];
            std::vector<int64_t> fill(P.flat_off.begin(), P.flat_off.end() - 1);
            P.flat_eid.resize(E);
            for (int64_t e = 0; e < E; ++e) P.flat_eid[fill[col[e]]++] = (int32_t)e;
        }
    }
    lap(2);

    // (4) colour the partitions greedily: lowest colour unused by any partition
    // already sharing one of its nodes.  Colours are handed out in rounds of 64
    // (one bit mask per node per round); a partition that finds all 64 colours
    // of a round taken waits for the next round.
    if (P.coloured_ok) {
        std::vector<uint64_t> nmask(N, 0);
        P.block_colour.assign(nb, -1);
        std::vector<int32_t> todo(nb), next;
        std::iota(todo.begin(), todo.end(), 0);
        int base = 0;
        while (!todo.empty()) {
            if (base >= kMaxBlockColours) {
                P.coloured_ok = false;
                P.coloured_why = "more than " + std::to_string(kMaxBlockColours) + " partition colours";
                break;
            }
            std::fill(nmask.begin(), nmask.end(), 0);
            next.clear();
            for (int32_t b : todo) {
                uint64_t used = 0;
                for (int64_t u = P.uniq_off[b]; u < P.uniq_off[b + 1]; ++u) used |= nmask[P.uniq[u]];
                int c = lowest_free(used);
                if (c < 0) {
                    next.push_back(b);
                    continue;
                }
                for (int64_t u = P.uniq_off[b]; u < P.uniq_off[b + 1]; ++u)
                    nmask[P.uniq[u]] |= 1ULL << c;
                P.block_colour[b] = base + c;
            }
            todo.swap(next);
            base += 64;
        }
    }
    if (P.coloured_ok) {
        const int nc = [&] {
            int m = 0;
            for (int32_t c : P.block_colour) m = std::max(m, c + 1);
            return m;
        }();
        P.nblock_colours = nc;
        P.colour_off.assign(nc + 1, 0);
        for (int64_t b = 0; b < nb; ++b) ++P.colour_off[P.block_colour[b] + 1];
        for (int c = 0; c < nc; ++c) P.colour_off[c + 1] += P.colour_off[c];
        P.colour_blocks.resize(nb);
        std::vector<int64_t> fill(P.colour_off.begin(), P.colour_off.end() - 1);
        for (int64_t b = 0; b < nb; ++b) P.colour_blocks[fill[P.block_colour[b]]++] = (int32_t)b;
        // a round may leave colours unused; drop them so every colour is non-empty
        std::vector<int64_t> off2(1, 0);
        std::vector<int32_t> remap(nc, -1);
        for (int c = 0; c < nc; ++c)
            if (P.colour_off[c + 1] > P.colour_off[c]) {
                remap[c] = (int32_t)off2.size() - 1;
                off2.push_back(P.colour_off[c + 1]);
            }
        for (int64_t b = 0; b < nb; ++b) P.block_colour[b] = remap[P.block_colour[b]];
        P.colour_off.swap(off2);
        P.nblock_colours = (int32_t)P.colour_off.size() - 1;
        P.min_blocks_per_colour = (int32_t)nb;
        for (int c = 0; c < P.nblock_colours; ++c)
            P.min_blocks_per_colour = std::min<int32_t>(
                P.min_blocks_per_colour, (int32_t)(P.colour_off[c + 1] - P.colour_off[c]));
    }
    if (!P.coloured_ok) {
        // the coloured variants are unavailable: drop their partial arrays
        P.block_colour.clear();
        P.colour_blocks.clear();
        P.colour_off.assign(1, 0);
        P.nblock_colours = 0;
        P.min_blocks_per_colour = 0;
        P.ecol.assign(E, 0);
        P.block_ncol.assign(nb, 0);
        P.uniq.clear();
        P.uniq_off.assign(nb + 1, 0);
        P.lidx.assign(2 * E, 0);
        P.max_elem_colours = 0;
        P.mean_elem_colours = 0.0;
        P.max_unique = 0;
    }
    lap(3);
    return OPF_OK;
}

VerifyResult verify_plan(const Plan &P, const int32_t *e2n_user)
{
    VerifyResult r;
    auto fail = [&](int prop, int64_t where, const std::string &msg) {
        r.ok = false;
        r.property = prop;
        r.where = where;
        r.message = msg;
        return r;
    };
    const int64_t N = P.N, E = P.E, nb = P.nblocks();
    // (1) node relabelling is a bijection
    if ((int64_t)P.node_new.size() != N) return fail(1, -1, "node relabelling has the wrong size");
    {
        std::vector<char> seen(N, 0);
        for (int64_t i = 0; i < N; ++i) {
            int32_t v = P.node_new[i];
            if (v < 0 || v >= N || seen[v]) return fail(1, i, "node relabelling is not a bijection");
            seen[v] = 1;
        }
    }
    // (2) edge reordering is a bijection that keeps endpoints and orientation
    if ((int64_t)P.edge_new.size() != E || (int64_t)P.e2n.size() != 2 * E)
        return fail(2, -1, "edge arrays have the wrong size");
    {
        std::vector<char> seen(E, 0);
        for (int64_t e = 0; e < E; ++e) {
            int32_t k = P.edge_new[e];
            if (k < 0 || k >= E || seen[k]) return fail(2, e, "edge reordering is not a bijection");
            seen[k] = 1;
            if (P.e2n[2 * k] != P.node_new[e2n_user[2 * e]] ||
                P.e2n[2 * k + 1] != P.node_new[e2n_user[2 * e + 1]])
                return fail(2, e, "internal map does not match the relabelled user map");
        }
    }
    // (5) partitions: contiguous, cover [0,E), at most block_size edges, grouped by colour
    if ((int64_t)P.block_off.size() != nb + 1 || P.block_off[0] != 0 || P.block_off[nb] != E)
        return fail(5, -1, "partition offsets do not cover the edge set");
    for (int64_t b = 0; b < nb; ++b) {
        int64_t n = P.block_off[b + 1] - P.block_off[b];
        if (n <= 0 || n > P.block_size) return fail(5, b, "partition size out of range");
    }
    // properties 3-7 hold for the two-level colouring, when the plan has one
    if (P.coloured_ok) {
        if ((int64_t)P.colour_off.size() != P.nblock_colours + 1 || P.colour_off[0] != 0 ||
            P.colour_off[P.nblock_colours] != nb || (int64_t)P.colour_blocks.size() != nb)
            return fail(5, -1, "colour offsets do not cover the partitions");
        {
            std::vector<char> seen(nb, 0);
            for (int c = 0; c < P.nblock_colours; ++c) {
                if (P.colour_off[c + 1] <= P.colour_off[c]) return fail(5, c, "empty partition colour");
                for (int64_t k = P.colour_off[c]; k < P.colour_off[c + 1]; ++k) {
                    int32_t b = P.colour_blocks[k];
                    if (b < 0 || b >= nb || seen[b] || P.block_colour[b] != c)
                        return fail(5, k, "partition listed under the wrong colour or twice");
                    seen[b] = 1;
                }
            }
        }
        // (7) colour counts fit their types
        if (P.nblock_colours < 1 || P.nblock_colours > kMaxBlockColours)
            return fail(7, -1, "partition colour count");
        for (int64_t b = 0; b < nb; ++b)
            if (P.block_ncol[b] < 1 || P.block_ncol[b] > 64) return fail(7, b, "edge colour count");
        // (6) local indices resolve to the map's nodes; unique lists sorted and distinct
        if ((int64_t)P.uniq_off.size() != nb + 1 || P.uniq_off[nb] != (int64_t)P.uniq.size())
            return fail(6, -1, "distinct-node offsets do not match the lists");
        for (int64_t b = 0; b < nb; ++b) {
            const int64_t u0 = P.uniq_off[b], nu = P.uniq_off[b + 1] - u0;
            if (nu < 1 || nu > 65535) return fail(7, b, "distinct-node count out of range");
            for (int64_t u = 1; u < nu; ++u)
                if (P.uniq[u0 + u] <= P.uniq[u0 + u - 1]) return fail(6, b, "distinct nodes not sorted");
            for (int64_t k = P.block_off[b]; k < P.block_off[b + 1]; ++k)
                for (int s = 0; s < 2; ++s) {
                    int64_t l = P.lidx[2 * k + s];
                    if (l >= nu || P.uniq[u0 + l] != P.e2n[2 * k + s])
                        return fail(6, k, "local index does not resolve to the map's node");
                }
            for (int64_t k = P.block_off[b]; k < P.block_off[b + 1]; ++k)
                if (P.ecol[k] >= P.block_ncol[b]) return fail(7, k, "edge colour above the count");
        }
        // (3) partitions of one colour share no node
        {
            std::vector<int32_t> stamp(N, -1);
            for (int c = 0; c < P.nblock_colours; ++c)
                for (int64_t k = P.colour_off[c]; k < P.colour_off[c + 1]; ++k) {
                    const int32_t b = P.colour_blocks[k];
                    for (int64_t u = P.uniq_off[b]; u < P.uniq_off[b + 1]; ++u) {
                        const int32_t v = P.uniq[u];
                        if (stamp[v] == c) return fail(3, b, "two partitions of one colour share a node");
                        stamp[v] = c;
                    }
                }
        }
        // (4) inside a partition, edges of one colour share no node
        {
            std::vector<uint64_t> lm;
            for (int64_t b = 0; b < nb; ++b) {
                lm.assign(P.uniq_off[b + 1] - P.uniq_off[b], 0);
                for (int64_t k = P.block_off[b]; k < P.block_off[b + 1]; ++k) {
                    uint64_t bit = 1ULL << P.ecol[k];
                    int li = P.lidx[2 * k], lj = P.lidx[2 * k + 1];
                    if ((lm[li] & bit) || (lm[lj] & bit) || li == lj)
                        return fail(4, k, "two edges of one colour share a node");
                    lm[li] |= bit;
                    lm[lj] |= bit;
                }
            }
        }
    }
    // (8) owner clusters: every edge is in the work of exactly the clusters of
    // its two endpoints (once when both are in one cluster)
    if (P.cluster_size > 0) {
        const int K = P.cluster_size;
        const int64_t ncl = P.nclusters();
        if ((int64_t)P.cl_seg_off.size() != ncl + 1 || P.cl_seg_off[0] != 0 ||
            P.cl_seg_off[ncl] != (int64_t)P.cl_seg_start.size())
            return fail(8, -1, "cluster segment offsets are inconsistent");
        std::vector<uint8_t> seen(E, 0);
        for (int64_t c = 0; c < ncl; ++c)
            for (int64_t s = P.cl_seg_off[c]; s < P.cl_seg_off[c + 1]; ++s) {
                const int64_t k0 = P.cl_seg_start[s], n = P.cl_seg_len[s];
                if (k0 < 0 || n < 1 || k0 + n > E) return fail(8, c, "segment outside the edge set");
                for (int64_t k = k0; k < k0 + n; ++k) {
                    const int64_t a = P.e2n[2 * k] / K, b = P.e2n[2 * k + 1] / K;
                    if (a != c && b != c) return fail(8, k, "edge listed for a cluster it does not touch");
                    if (seen[k] == 255) return fail(8, k, "edge listed too often");
                    ++seen[k];
                }
            }
        for (int64_t k = 0; k < E; ++k) {
            const int want = (P.e2n[2 * k] / K == P.e2n[2 * k + 1] / K) ? 1 : 2;
            if (seen[k] != want) return fail(8, k, "edge missing from its clusters' work");
        }
        // the visit lists hold the same work
        if ((int64_t)P.cl_prim.size() != 2 * ncl || (int64_t)P.cl_sec_off.size() != ncl + 1 ||
            P.cl_sec_off[0] != 0 || P.cl_sec_off[ncl] != (int64_t)P.cl_sec_eid.size())
            return fail(8, -1, "cluster visit lists are inconsistent");
        std::fill(seen.begin(), seen.end(), 0);
        auto visit = [&](int64_t c, int64_t k) -> bool {
            if (k < 0 || k >= E) return false;
            const int64_t a = P.e2n[2 * k] / K, b = P.e2n[2 * k + 1] / K;
            if ((a != c && b != c) || seen[k] == 255) return false;
            ++seen[k];
            return true;
        };
        for (int64_t c = 0; c < ncl; ++c) {
            const int64_t p0 = P.cl_prim[2 * c], pn = P.cl_prim[2 * c + 1];
            if (pn < 0) return fail(8, c, "negative visit range");
            for (int64_t k = p0; k < p0 + pn; ++k)
                if (!visit(c, k)) return fail(8, k, "visit range holds an edge of another cluster");
            for (int64_t s = P.cl_sec_off[c]; s < P.cl_sec_off[c + 1]; ++s)
                if (!visit(c, P.cl_sec_eid[s])) return fail(8, s, "visit list holds an edge of another cluster");
        }
        for (int64_t k = 0; k < E; ++k) {
            const int want = (P.e2n[2 * k] / K == P.e2n[2 * k + 1] / K) ? 1 : 2;
            if (seen[k] != want) return fail(8, k, "edge missing from its clusters' visit lists");
        }
        // the two loops of the owner kernel cover every end of every edge exactly
        // once: interior blocks both ends, each cut visit the end it names (in
        // both orders of the cut visits)
        if ((int64_t)P.cl_nint.size() != ncl || (int64_t)P.cl_cut_off.size() != ncl + 1 ||
            P.cl_cut_off[0] != 0 || P.cl_cut_off[ncl] != (int64_t)P.cl_cut_eid.size() ||
            P.cl_cut_eid.size() != P.cl_cut_end.size() || P.cl_cutf_eid.size() != P.cl_cut_eid.size() ||
            P.cl_cutf_end.size() != P.cl_cut_eid.size())
            return fail(8, -1, "interior blocks or cut visits are inconsistent");
        for (int order = 0; order < 2; ++order) {
            const std::vector<int32_t> &ce = order ? P.cl_cutf_eid : P.cl_cut_eid;
            const std::vector<uint8_t> &ch = order ? P.cl_cutf_end : P.cl_cut_end;
            std::vector<uint8_t> ends(E, 0);  // bit h: end h covered
            for (int64_t c = 0; c < ncl; ++c) {
                const int64_t p0 = P.cl_prim[2 * c], ni = P.cl_nint[c];
                if (ni < 0 || ni > P.cl_prim[2 * c + 1]) return fail(8, c, "interior block outside the range");
                for (int64_t k = p0; k < p0 + ni; ++k) {
                    if (P.e2n[2 * k] / K != c || P.e2n[2 * k + 1] / K != c)
                        return fail(8, k, "interior block holds an edge with an end outside the cluster");
                    if (ends[k]) return fail(8, k, "edge end covered twice");
                    ends[k] = 3;
                }
                for (int64_t s = P.cl_cut_off[c]; s < P.cl_cut_off[c + 1]; ++s) {
                    const int64_t k = ce[s];
                    const int h = ch[s];
                    if (k < 0 || k >= E || h > 1) return fail(8, s, "cut visit out of range");
                    if (P.e2n[2 * k + h] / K != c) return fail(8, s, "cut visit names an end outside the cluster");
                    if (ends[k] & (1 << h)) return fail(8, k, "edge end covered twice");
                    ends[k] |= (uint8_t)(1 << h);
                }
            }
            for (int64_t k = 0; k < E; ++k)
                if (ends[k] != 3) return fail(8, k, "edge end missing from the owner kernel's loops");
        }
    }
    // (9) flat colouring: every edge in exactly one colour; edges of one colour
    // share no node
    if (P.flat_ok) {
        const int nc = P.flat_colours;
        if (nc < 1 || nc > 128 || (int64_t)P.flat_off.size() != nc + 1 || P.flat_off[0] != 0 ||
            P.flat_off[nc] != E || (int64_t)P.flat_eid.size() != E)
            return fail(9, -1, "flat colour offsets are inconsistent");
        std::vector<uint8_t> seen(E, 0);
        std::vector<int32_t> stamp(N, -1);
        for (int c = 0; c < nc; ++c) {
            if (P.flat_off[c + 1] <= P.flat_off[c]) return fail(9, c, "empty flat colour");
            for (int64_t s = P.flat_off[c]; s < P.flat_off[c + 1]; ++s) {
                const int64_t k = P.flat_eid[s];
                if (k < 0 || k >= E || seen[k]) return fail(9, k, "edge listed twice or out of range");
                seen[k] = 1;
                const int32_t a = P.e2n[2 * k], b = P.e2n[2 * k + 1];
                if (stamp[a] == c || stamp[b] == c) return fail(9, k, "two edges of one flat colour share a node");
                stamp[a] = stamp[b] = c;
            }
        }
    }
    return r;
}

}  // namespace opf
