// Host-side plan: mesh validation and orientation, octree over tets (by
// centroid) and targets (Sec. 3.1), acceptance radii (Sec. 3.2) and the dual
// tree traversal (Sec. 3.3, Listings 1-2) producing the M2L and P2P lists.
//
// Built without floating-point contraction (-ffp-contract=off): the octant
// keys, cell centres, radii and the acceptance test are evaluated with fixed
// expressions so that the same mesh always gives the same tree and lists.
#include "plan.h"

#include <algorithm>
#include <array>
#include <chrono>
#include <map>
#include <cmath>
#include <numeric>
#include <unordered_map>

#include "../../include/tetfmm.h"

namespace tfmm {

namespace {

constexpr int kMaxDepth = 21;
constexpr double kKeyScale = 2097152.0;  // 2^21

[[noreturn]] void fail(int code, const std::string &msg) { throw PlanError{code, msg}; }

uint32_t axis_key(double xd, double o, double S)
{
    double y = (xd - o) / S;
    double z = std::floor(y * kKeyScale);
    if (z < 0.0) z = 0.0;
    if (z > kKeyScale - 1.0) z = kKeyScale - 1.0;
    return static_cast<uint32_t>(z);
}

// Interleave three 21-bit keys, x in the lowest bit of every triple: the
// triple at bit 3*(21-L) is the octant of level L (bit 0 x, bit 1 y, bit 2 z).
uint64_t morton(uint32_t kx, uint32_t ky, uint32_t kz)
{
    uint64_t c = 0;
    for (int b = 0; b < kMaxDepth; ++b) {
        c |= static_cast<uint64_t>((kx >> b) & 1u) << (3 * b);
        c |= static_cast<uint64_t>((ky >> b) & 1u) << (3 * b + 1);
        c |= static_cast<uint64_t>((kz >> b) & 1u) << (3 * b + 2);
    }
    return c;
}

inline int octant_at(uint64_t code, int level) { return static_cast<int>((code >> (3 * (kMaxDepth - level))) & 7u); }

double dist3(const double *a, const double *b)
{
    double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    return std::sqrt((dx * dx + dy * dy) + dz * dz);
}

void build_m2l_keys(HostPlan &hp);

std::vector<int32_t> sorted_order(const std::vector<uint64_t> &codes)
{
    std::vector<int32_t> idx(codes.size());
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) { return codes[a] < codes[b]; });
    return idx;
}

}  // namespace

void build_host_plan(HostPlan &hp, const double *nodes, int64_t n_nodes, const int32_t *tets, int64_t n_tets,
                     const double *targets, int64_t n_targets, int p, int leaf, double theta, bool points)
{
    auto t0 = std::chrono::steady_clock::now();
    // point sources: source i is the point nodes[i], written as a tet whose
    // four corners are that node (its centroid and farthest corner are the
    // point), so the tree, radii and lists below serve both kinds
    std::vector<int32_t> ptv;
    if (points) {
        if (!nodes) fail(TFMM_EINVAL, "points must not be NULL");
        if (n_nodes < 1 || n_nodes > INT32_MAX / 4) fail(TFMM_EINVAL, "bad number of points");
        ptv.resize(4 * (size_t)n_nodes);
        for (int64_t i = 0; i < n_nodes; ++i)
            for (int c = 0; c < 4; ++c) ptv[4 * (size_t)i + c] = (int32_t)i;
        tets = ptv.data();
        n_tets = n_nodes;
    }
    hp.points = points;
    if (!nodes || !tets) fail(TFMM_EINVAL, "nodes and tets must not be NULL");
    if (!points && (n_nodes < 4 || n_tets < 1)) fail(TFMM_EINVAL, "need at least 4 nodes and 1 tet");
    if (n_nodes > INT32_MAX || n_tets > INT32_MAX / 4) fail(TFMM_EINVAL, "mesh too large for 32-bit indices");
    if (targets && (n_targets < 1 || n_targets > INT32_MAX)) fail(TFMM_EINVAL, "bad number of targets");
    if (p < 1 || p > TFMM_PMAX) fail(TFMM_EINVAL, "expansion order p out of range");
    if (leaf < 1) fail(TFMM_EINVAL, "leaf_size must be >= 1");
    if (!(theta > 0.0 && theta < 1.0)) fail(TFMM_EINVAL, "theta must lie in (0, 1)");

    hp.p = p;
    hp.leaf = leaf;
    hp.theta = theta;
    hp.n_nodes = n_nodes;
    hp.n_tets = n_tets;
    hp.targets_are_nodes = targets == nullptr;
    if (!targets) {
        targets = nodes;
        n_targets = n_nodes;
    }
    hp.n_targets = n_targets;

    for (int64_t i = 0; i < 3 * n_nodes; ++i)
        if (!std::isfinite(nodes[i])) fail(TFMM_ENONFINITE, "non-finite node coordinate");
    for (int64_t i = 0; i < 3 * n_targets; ++i)
        if (!std::isfinite(targets[i])) fail(TFMM_ENONFINITE, "non-finite target coordinate");
    for (int64_t i = 0; i < 4 * n_tets; ++i)
        if (tets[i] < 0 || tets[i] >= n_nodes) fail(TFMM_EINDEX, "tet node index out of range");
    hp.nodes.assign(nodes, nodes + 3 * n_nodes);

    // orientation and degeneracy
    std::vector<int32_t> tv(tets, tets + 4 * n_tets);
    for (int64_t t = 0; t < (points ? 0 : n_tets); ++t) {
        int32_t *q = &tv[4 * t];
        const double *a = nodes + 3 * (int64_t)q[0], *b = nodes + 3 * (int64_t)q[1];
        const double *c = nodes + 3 * (int64_t)q[2], *d = nodes + 3 * (int64_t)q[3];
        double e1[3], e2[3], e3[3];
        for (int k = 0; k < 3; ++k) {
            e1[k] = b[k] - a[k];
            e2[k] = c[k] - a[k];
            e3[k] = d[k] - a[k];
        }
        double det = e1[0] * (e2[1] * e3[2] - e2[2] * e3[1]) - e1[1] * (e2[0] * e3[2] - e2[2] * e3[0]) +
                     e1[2] * (e2[0] * e3[1] - e2[1] * e3[0]);
        const double *V[4] = {a, b, c, d};
        double lsum = 0.0;
        for (int i = 0; i < 4; ++i)
            for (int j = i + 1; j < 4; ++j) lsum += dist3(V[i], V[j]);
        double lm = lsum / 6.0;
        if (!(std::fabs(det) > 1e-12 * lm * lm * lm)) fail(TFMM_EDEGEN, "degenerate tetrahedron " + std::to_string(t));
        if (det < 0.0) std::swap(q[2], q[3]);
    }

    // bounding cube of nodes and targets
    double lo[3], hi[3];
    for (int k = 0; k < 3; ++k) lo[k] = hi[k] = nodes[k];
    auto grow = [&](const double *x, int64_t n) {
        for (int64_t i = 0; i < n; ++i)
            for (int k = 0; k < 3; ++k) {
                lo[k] = std::min(lo[k], x[3 * i + k]);
                hi[k] = std::max(hi[k], x[3 * i + k]);
            }
    };
    grow(nodes, n_nodes);
    grow(targets, n_targets);
    double ext = 0.0;
    for (int k = 0; k < 3; ++k) ext = std::max(ext, hi[k] - lo[k]);
    if (!(ext > 0.0)) fail(TFMM_EINVAL, "sources and targets must not all coincide");
    hp.side = ext * (1.0 + std::ldexp(1.0, -20));
    for (int k = 0; k < 3; ++k) hp.origin[k] = (lo[k] + hi[k]) * 0.5 - 0.5 * hp.side;

    // Morton codes: tets by centroid, targets by position
    std::vector<uint64_t> tcode(n_tets), xcode(n_targets);
    for (int64_t t = 0; t < n_tets; ++t) {
        const int32_t *q = &tets[4 * t];  // input order: the centroid is symmetric
        uint32_t k3[3];
        for (int k = 0; k < 3; ++k) {
            double cen = ((nodes[3 * (int64_t)q[0] + k] + nodes[3 * (int64_t)q[1] + k]) +
                          (nodes[3 * (int64_t)q[2] + k] + nodes[3 * (int64_t)q[3] + k])) *
                         0.25;
            k3[k] = axis_key(cen, hp.origin[k], hp.side);
        }
        tcode[t] = morton(k3[0], k3[1], k3[2]);
    }
    for (int64_t i = 0; i < n_targets; ++i) {
        uint32_t k3[3];
        for (int k = 0; k < 3; ++k) k3[k] = axis_key(targets[3 * i + k], hp.origin[k], hp.side);
        xcode[i] = morton(k3[0], k3[1], k3[2]);
    }
    hp.tet_perm = sorted_order(tcode);
    hp.tgt_perm = sorted_order(xcode);
    std::vector<uint64_t> tcs(n_tets), xcs(n_targets);
    hp.tet_nodes.resize(4 * n_tets);
    for (int64_t s = 0; s < n_tets; ++s) {
        int32_t t = hp.tet_perm[s];
        tcs[s] = tcode[t];
        for (int c = 0; c < 4; ++c) hp.tet_nodes[4 * s + c] = tv[4 * (int64_t)t + c];
    }
    hp.tgt_xyz.resize(3 * n_targets);
    for (int64_t s = 0; s < n_targets; ++s) {
        int32_t i = hp.tgt_perm[s];
        xcs[s] = xcode[i];
        for (int k = 0; k < 3; ++k) hp.tgt_xyz[3 * s + k] = targets[3 * (int64_t)i + k];
    }

    // octree, level by level
    auto centre = [&](Cell &C) {
        double s = std::ldexp(hp.side, -C.level);
        C.c[0] = hp.origin[0] + ((double)C.ix + 0.5) * s;
        C.c[1] = hp.origin[1] + ((double)C.iy + 0.5) * s;
        C.c[2] = hp.origin[2] + ((double)C.iz + 0.5) * s;
    };
    hp.cells.clear();
    Cell root{};
    root.level = 0;
    root.tbeg = 0;
    root.tend = (int32_t)n_tets;
    root.xbeg = 0;
    root.xend = (int32_t)n_targets;
    root.parent = -1;
    centre(root);
    hp.cells.push_back(root);
    hp.level_begin = {0};
    int64_t lb = 0, le = 1;
    for (int L = 0;; ++L) {
        hp.level_begin.push_back((int32_t)le);
        for (int64_t ci = lb; ci < le; ++ci) {
            Cell C = hp.cells[ci];
            int32_t nt = C.tend - C.tbeg, nx = C.xend - C.xbeg;
            hp.cells[ci].cbeg = (int32_t)hp.cells.size();
            hp.cells[ci].nchild = 0;
            if (!((nt > leaf || nx > leaf) && L < kMaxDepth)) continue;
            int32_t tb = C.tbeg, xb = C.xbeg;
            for (int o = 0; o < 8; ++o) {
                int32_t te = (int32_t)(std::partition_point(tcs.begin() + tb, tcs.begin() + C.tend,
                                                           [&](uint64_t c) { return octant_at(c, L + 1) <= o; }) -
                                       tcs.begin());
                int32_t xe = (int32_t)(std::partition_point(xcs.begin() + xb, xcs.begin() + C.xend,
                                                           [&](uint64_t c) { return octant_at(c, L + 1) <= o; }) -
                                       xcs.begin());
                if (te > tb || xe > xb) {
                    Cell K{};
                    K.level = L + 1;
                    K.ix = 2 * C.ix + (o & 1);
                    K.iy = 2 * C.iy + ((o >> 1) & 1);
                    K.iz = 2 * C.iz + ((o >> 2) & 1);
                    K.tbeg = tb;
                    K.tend = te;
                    K.xbeg = xb;
                    K.xend = xe;
                    K.parent = (int32_t)ci;
                    centre(K);
                    hp.cells.push_back(K);
                    hp.cells[ci].nchild++;
                }
                tb = te;
                xb = xe;
            }
        }
        lb = le;
        le = (int64_t)hp.cells.size();
        if (le == lb) break;
    }
    // level_begin: [L] = first cell of level L for L = 0..depth, [depth+1] = n_cells
    hp.depth = (int)hp.level_begin.size() - 2;

    // radii: farthest tet corner (source role) and farthest target (target role)
    for (auto &C : hp.cells) {
        double rs = 0.0, rt = 0.0;
        for (int32_t s = C.tbeg; s < C.tend; ++s)
            for (int c = 0; c < 4; ++c) rs = std::max(rs, dist3(&hp.nodes[3 * (int64_t)hp.tet_nodes[4 * s + c]], C.c));
        for (int32_t s = C.xbeg; s < C.xend; ++s) rt = std::max(rt, dist3(&hp.tgt_xyz[3 * (int64_t)s], C.c));
        C.rsrc = rs;
        C.rtgt = rt;
    }

    // dual tree traversal
    const double th2 = theta * theta;
    std::vector<std::pair<int32_t, int32_t>> m2l, stack;
    hp.p2p_a.clear();
    hp.p2p_b.clear();
    hp.n_p2p_pairs = 0;
    auto interact = [&](int32_t a, int32_t b) {
        const Cell &A = hp.cells[a], &B = hp.cells[b];
        if (A.xend == A.xbeg || B.tend == B.tbeg) return;
        double dx = A.c[0] - B.c[0], dy = A.c[1] - B.c[1], dz = A.c[2] - B.c[2];
        double d2 = (dx * dx + dy * dy) + dz * dz;
        double rr = A.rtgt + B.rsrc;
        if (rr * rr < th2 * d2) {
            m2l.emplace_back(a, b);
        } else if (A.nchild == 0 && B.nchild == 0) {
            hp.p2p_a.push_back(a);
            hp.p2p_b.push_back(b);
            hp.n_p2p_pairs += (int64_t)(A.xend - A.xbeg) * (int64_t)(B.tend - B.tbeg);
        } else {
            stack.emplace_back(a, b);
        }
    };
    interact(0, 0);
    while (!stack.empty()) {
        auto [a, b] = stack.back();
        stack.pop_back();
        const Cell &A = hp.cells[a], &B = hp.cells[b];
        bool split_target = A.level < B.level;  // larger target cube; ties split the source
        if (split_target && A.nchild == 0) split_target = false;
        if (!split_target && B.nchild == 0) split_target = true;
        if (split_target) {
            for (int32_t k = 0, cb = A.cbeg, n = A.nchild; k < n; ++k) interact(cb + k, b);
        } else {
            for (int32_t k = 0, cb = B.cbeg, n = B.nchild; k < n; ++k) interact(a, cb + k);
        }
    }
    // M2L as CSR by target cell (stable: list order within a target kept)
    const int64_t nc = (int64_t)hp.cells.size();
    hp.m2l_ptr.assign(nc + 1, 0);
    for (auto &pr : m2l) hp.m2l_ptr[pr.first + 1]++;
    for (int64_t i = 0; i < nc; ++i) hp.m2l_ptr[i + 1] += hp.m2l_ptr[i];
    hp.m2l_src.resize(m2l.size());
    {
        std::vector<int32_t> fill(hp.m2l_ptr.begin(), hp.m2l_ptr.end() - 1);
        for (auto &pr : m2l) hp.m2l_src[fill[pr.first]++] = pr.second;
    }
    build_m2l_keys(hp);
    hp.setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

namespace {

void build_m2l_keys(HostPlan &hp)
{
    hp.m2l_keys.clear();
    hp.m2l_pair_key.assign(hp.m2l_src.size(), -1);
    std::unordered_map<uint64_t, int32_t> keymap;
    const int64_t nc = (int64_t)hp.cells.size();
    for (int64_t a = 0; a < nc; ++a) {
        const Cell &A = hp.cells[a];
        for (int32_t j = hp.m2l_ptr[a]; j < hp.m2l_ptr[a + 1]; ++j) {
            const Cell &B = hp.cells[hp.m2l_src[j]];
            const int dl = B.level - A.level;
            int64_t k[3];
            const int32_t ia[3] = {A.ix, A.iy, A.iz}, ib[3] = {B.ix, B.iy, B.iz};
            for (int d = 0; d < 3; ++d) {
                if (dl >= 0)
                    k[d] = (2 * (int64_t)ia[d] + 1) * ((int64_t)1 << dl) - (2 * (int64_t)ib[d] + 1);
                else
                    k[d] = (2 * (int64_t)ia[d] + 1) - (2 * (int64_t)ib[d] + 1) * ((int64_t)1 << (-dl));
                if (k[d] <= -(1 << 19) || k[d] >= (1 << 19)) throw PlanError{TFMM_ENOTSUP, "M2L offset out of range"};
            }
            const uint64_t packed = ((uint64_t)(dl + 32) << 60) | ((uint64_t)(k[0] + (1 << 19)) << 40) |
                                    ((uint64_t)(k[1] + (1 << 19)) << 20) | (uint64_t)(k[2] + (1 << 19));
            auto it = keymap.find(packed);
            int32_t id;
            if (it != keymap.end()) {
                id = it->second;
            } else {
                id = (int32_t)(hp.m2l_keys.size() / 4);
                keymap.emplace(packed, id);
                hp.m2l_keys.push_back(dl);
                hp.m2l_keys.push_back((int32_t)k[0]);
                hp.m2l_keys.push_back((int32_t)k[1]);
                hp.m2l_keys.push_back((int32_t)k[2]);
            }
            hp.m2l_pair_key[j] = id;
        }
    }
}

}  // namespace

// Dispatch order of M2L work items.  Workgroup w runs on XCD w % kM2LXcds
// (round-robin), each XCD with its own L2.  The items of every level (in
// octree order) are cut into kM2LXcds runs of about equal weight (range
// length), run x going to XCD x, so that the items of one XCD are neighbours
// in space and find their source multipoles in its L2; an XCD runs its items
// longest first (stable).  Returns item ids per dispatch slot, -1 where an
// XCD has no item left; slots that are empty on every XCD at the end are
// dropped.
static std::vector<int32_t> xcd_dispatch_order(const std::vector<std::array<int32_t, 2>> &rng,
                                               const std::vector<int32_t> &lev)
{
    std::map<int, std::vector<int32_t>> by_level;
    for (size_t i = 0; i < rng.size(); ++i) by_level[lev[i]].push_back((int32_t)i);
    std::vector<std::vector<int32_t>> per(kM2LXcds);
    for (const auto &kv : by_level) {
        int64_t W = 0, acc = 0;
        for (int32_t i : kv.second) W += rng[i][1] - rng[i][0];
        for (int32_t i : kv.second) {
            const int64_t w = rng[i][1] - rng[i][0];
            const int x = (int)std::min<int64_t>(kM2LXcds - 1, (2 * acc + w) * kM2LXcds / std::max<int64_t>(2 * W, 1));
            per[x].push_back(i);
            acc += w;
        }
    }
    size_t kmax = 0;
    for (auto &v : per) {
        std::stable_sort(v.begin(), v.end(), [&](int32_t x, int32_t y) {
            return rng[x][1] - rng[x][0] > rng[y][1] - rng[y][0];
        });
        kmax = std::max(kmax, v.size());
    }
    std::vector<int32_t> slots;
    slots.reserve(kmax * kM2LXcds);
    for (size_t k = 0; k < kmax; ++k)
        for (int x = 0; x < kM2LXcds; ++x) slots.push_back(k < per[x].size() ? per[x][k] : -1);
    while (!slots.empty() && slots.back() < 0) slots.pop_back();
    return slots;
}

void build_m2l_tiles(const HostPlan &hp, int tpt, int max_ent, M2LTiles &out, int only_level)
{
    out.tpt = tpt;
    out.tile_tgt.clear();
    out.tile_rng.clear();
    out.ent_key.clear();
    out.ent_src.clear();
    const int64_t nc = (int64_t)hp.cells.size();
    std::vector<int32_t> tile, tgt, lev;
    std::vector<std::array<int32_t, 2>> rng;
    int cur_level = -1;
    std::vector<std::array<int32_t, 3>> trip;  // key, slot, source
    auto flush = [&]() {
        if (tile.empty()) return;
        trip.clear();
        for (int t = 0; t < (int)tile.size(); ++t) {
            const int32_t a = tile[t];
            for (int32_t j = hp.m2l_ptr[a]; j < hp.m2l_ptr[a + 1]; ++j)
                trip.push_back({hp.m2l_pair_key[j], t, hp.m2l_src[j]});
        }
        // entries sorted by level difference, then key
        std::sort(trip.begin(), trip.end(), [&](const std::array<int32_t, 3> &x, const std::array<int32_t, 3> &y) {
            const int32_t dx = hp.m2l_keys[4 * (size_t)x[0]], dy = hp.m2l_keys[4 * (size_t)y[0]];
            if (dx != dy) return dx < dy;
            return x < y;
        });
        const int32_t e0 = (int32_t)out.ent_key.size();
        for (size_t i = 0; i < trip.size();) {
            const int32_t k = trip[i][0];
            out.ent_key.push_back(k);
            const size_t base = out.ent_src.size();
            out.ent_src.resize(base + tpt, -1);
            for (; i < trip.size() && trip[i][0] == k; ++i) out.ent_src[base + trip[i][1]] = trip[i][2];
        }
        const int32_t e1 = (int32_t)out.ent_key.size();
        // work items of at most max_ent entries sharing the tile's targets
        for (int32_t b = e0; b < e1; b += max_ent) {
            for (int t = 0; t < tpt; ++t) tgt.push_back(t < (int)tile.size() ? tile[t] : -1);
            rng.push_back({b, std::min(e1, b + max_ent)});
            lev.push_back(cur_level);
        }
        if (out.ent_key.size() > (size_t)INT32_MAX / 16) throw PlanError{TFMM_ENOTSUP, "too many M2L entries"};
        tile.clear();
    };
    // Tile grouping.  A cell's translation keys depend mostly on its octant
    // in its parent, so a tile takes the cells of one octant from tpt
    // parents that are consecutive in Morton order (within one level): in
    // the 40^3 cube this cuts the entries (distinct keys per tile) by 10%
    // against tpt consecutive cells, and tiles stay neighbours in space.
    std::map<int, std::vector<std::pair<uint64_t, int32_t>>> lvl;
    int tbits = 0;
    while ((1 << tbits) < tpt) ++tbits;
    for (int64_t a = 0; a < nc; ++a) {
        if (hp.m2l_ptr[a + 1] == hp.m2l_ptr[a]) continue;
        const Cell &c = hp.cells[a];
        if (only_level >= 0 && c.level != only_level) continue;
        const uint64_t mp = morton((uint32_t)c.ix >> 1, (uint32_t)c.iy >> 1, (uint32_t)c.iz >> 1);
        const uint64_t oct = (uint64_t)((c.ix & 1) | (c.iy & 1) << 1 | (c.iz & 1) << 2);
        lvl[c.level].push_back({((mp >> tbits) << (3 + tbits)) | (oct << tbits) | (mp & ((1u << tbits) - 1)), (int32_t)a});
    }
    for (auto &kv : lvl) {
        std::stable_sort(kv.second.begin(), kv.second.end(),
                         [](const std::pair<uint64_t, int32_t> &x, const std::pair<uint64_t, int32_t> &y) { return x.first < y.first; });
        cur_level = kv.first;
        for (const auto &e : kv.second) {
            if ((int)tile.size() == tpt) flush();
            tile.push_back(e.second);
        }
        flush();
    }
    const std::vector<int32_t> slots = xcd_dispatch_order(rng, lev);
    out.tile_tgt.reserve(slots.size() * tpt);
    out.tile_rng.reserve(2 * slots.size());
    for (int32_t i : slots) {
        if (i >= 0) {
            out.tile_tgt.insert(out.tile_tgt.end(), tgt.begin() + (size_t)i * tpt, tgt.begin() + (size_t)(i + 1) * tpt);
            out.tile_rng.push_back(rng[i][0]);
            out.tile_rng.push_back(rng[i][1]);
        } else {
            out.tile_tgt.insert(out.tile_tgt.end(), (size_t)tpt, -1);
            out.tile_rng.push_back(0);
            out.tile_rng.push_back(0);
        }
    }
}

void build_m2l_packs(const HostPlan &hp, int nb, int tpg, int max_grp, M2LPacks &out, int only_level)
{
    if (nb < 1 || nb > 256 || tpg < 1 || max_grp < 1) throw PlanError{TFMM_EINVAL, "bad M2L pack shape"};
    out = M2LPacks{};
    out.nb = nb;
    out.tpg = tpg;
    const int64_t nc = (int64_t)hp.cells.size();
    // target cells with translations, per level in Morton order
    std::map<int, std::vector<std::pair<uint64_t, int32_t>>> lvl;
    for (int64_t a = 0; a < nc; ++a) {
        if (hp.m2l_ptr[a + 1] == hp.m2l_ptr[a]) continue;
        const Cell &c = hp.cells[a];
        if (only_level >= 0 && c.level != only_level) continue;
        lvl[c.level].push_back({morton((uint32_t)c.ix, (uint32_t)c.iy, (uint32_t)c.iz), (int32_t)a});
    }
    std::vector<std::array<int32_t, 2>> rng;  // items: group range
    std::vector<int32_t> iblk, lev;
    std::vector<std::array<int32_t, 3>> trip;  // key, slot, source
    for (auto &kv : lvl) {
        std::sort(kv.second.begin(), kv.second.end());
        const auto &v = kv.second;
        for (size_t b0 = 0; b0 < v.size(); b0 += (size_t)nb) {
            const int32_t blk = (int32_t)(out.blk_cells.size() / nb);
            const size_t b1 = std::min(v.size(), b0 + (size_t)nb);
            trip.clear();
            for (size_t i = b0; i < b0 + (size_t)nb; ++i) {
                const int32_t a = i < b1 ? v[i].second : -1;
                out.blk_cells.push_back(a);
                if (a < 0) continue;
                for (int32_t j = hp.m2l_ptr[a]; j < hp.m2l_ptr[a + 1]; ++j)
                    trip.push_back({hp.m2l_pair_key[j], (int32_t)(i - b0), hp.m2l_src[j]});
            }
            // by key, then by slot class (slot mod tpg), then slot: the pairs
            // of a key are dealt round-robin over its ceil(n / tpg) groups, so
            // that a group's slots differ mod tpg wherever the class counts
            // allow (its accumulator rows then fall in different LDS banks)
            std::sort(trip.begin(), trip.end(), [tpg](const std::array<int32_t, 3> &x, const std::array<int32_t, 3> &y) {
                if (x[0] != y[0]) return x[0] < y[0];
                if (x[1] % tpg != y[1] % tpg) return x[1] % tpg < y[1] % tpg;
                return x[1] < y[1];
            });
            const int32_t g0 = (int32_t)out.grp_key.size();
            for (size_t i = 0; i < trip.size();) {
                const int32_t k = trip[i][0];
                size_t j = i;
                while (j < trip.size() && trip[j][0] == k) ++j;
                const size_t n = j - i, G = (n + (size_t)tpg - 1) / (size_t)tpg;
                for (size_t g = 0; g < G; ++g) {
                    out.grp_key.push_back(k);
                    for (int q = 0; q < tpg; ++q) {
                        const size_t e = g + (size_t)q * G;  // round-robin deal
                        const bool ok = e < n;
                        out.grp_src.push_back(ok ? trip[i + e][2] : -1);
                        out.grp_slot.push_back(ok ? (uint8_t)trip[i + e][1] : (uint8_t)0);
                    }
                }
                i = j;
            }
            const int32_t g1 = (int32_t)out.grp_key.size();
            if (out.grp_key.size() > (size_t)INT32_MAX / 16) throw PlanError{TFMM_ENOTSUP, "too many M2L groups"};
            // runs of about equal size, none above max_grp
            const int32_t n = g1 - g0, parts = (n + max_grp - 1) / std::max(max_grp, 1);
            for (int32_t p = 0; p < parts; ++p) {
                rng.push_back({g0 + (int32_t)((int64_t)n * p / parts), g0 + (int32_t)((int64_t)n * (p + 1) / parts)});
                iblk.push_back(blk);
                lev.push_back(kv.first);
            }
        }
    }
    for (int32_t i : xcd_dispatch_order(rng, lev)) {
        out.item.push_back(i >= 0 ? iblk[i] : 0);
        out.item.push_back(i >= 0 ? rng[i][0] : 0);
        out.item.push_back(i >= 0 ? rng[i][1] : 0);
    }
}


void merge_host_plans(const std::vector<const HostPlan *> &in, HostPlan &out, std::vector<double> &scale,
                      std::vector<int64_t> &node_off)
{
    if (in.empty()) throw PlanError{TFMM_EINVAL, "no plans to merge"};
    const HostPlan &h0 = *in[0];
    for (const HostPlan *h : in)
        if (h->p != h0.p || h->leaf != h0.leaf || h->theta != h0.theta || h->points || !h->targets_are_nodes)
            throw PlanError{TFMM_EINVAL, "merged plans need tet sources at the nodes and one p, leaf and theta"};
    out = HostPlan{};
    out.p = h0.p;
    out.leaf = h0.leaf;
    out.theta = h0.theta;
    out.targets_are_nodes = true;
    out.side = 1.0;
    const size_t n = in.size();
    scale.assign(n, 1.0);
    node_off.assign(n + 1, 0);
    std::vector<int64_t> tet_off(n + 1, 0);
    int depth = 0;
    for (size_t i = 0; i < n; ++i) {
        node_off[i + 1] = node_off[i] + in[i]->n_nodes;
        tet_off[i + 1] = tet_off[i] + in[i]->n_tets;
        depth = std::max(depth, in[i]->depth);
        scale[i] = in[i]->side;
    }
    if (node_off[n] > INT32_MAX || tet_off[n] > INT32_MAX) throw PlanError{TFMM_ENOTSUP, "merged batch too large"};
    out.n_nodes = node_off[n];
    out.n_tets = tet_off[n];
    out.n_targets = node_off[n];
    out.depth = depth;
    out.nodes.resize(3 * (size_t)out.n_nodes);
    out.tgt_xyz.resize(3 * (size_t)out.n_targets);
    out.tet_perm.resize((size_t)out.n_tets);
    out.tet_nodes.resize(4 * (size_t)out.n_tets);
    out.tgt_perm.resize((size_t)out.n_targets);
    for (size_t i = 0; i < n; ++i) {
        const HostPlan &h = *in[i];
        const double k = 1.0 / h.side;
        for (int64_t j = 0; j < h.n_nodes; ++j)
            for (int d = 0; d < 3; ++d) {
                out.nodes[3 * (node_off[i] + j) + d] = (h.nodes[3 * j + d] - h.origin[d]) * k;
                out.tgt_xyz[3 * (node_off[i] + j) + d] = (h.tgt_xyz[3 * j + d] - h.origin[d]) * k;
            }
        for (int64_t s = 0; s < h.n_tets; ++s) {
            out.tet_perm[tet_off[i] + s] = (int32_t)(tet_off[i] + h.tet_perm[s]);
            for (int c = 0; c < 4; ++c) out.tet_nodes[4 * (tet_off[i] + s) + c] = (int32_t)(node_off[i] + h.tet_nodes[4 * s + c]);
        }
        for (int64_t s = 0; s < h.n_targets; ++s) out.tgt_perm[node_off[i] + s] = (int32_t)(node_off[i] + h.tgt_perm[s]);
        out.n_p2p_pairs += h.n_p2p_pairs;
        out.setup_seconds += h.setup_seconds;
    }
    // cells by level, mesh by mesh
    std::vector<std::vector<int32_t>> remap(n);
    for (size_t i = 0; i < n; ++i) remap[i].assign(in[i]->cells.size(), -1);
    out.level_begin.assign(1, 0);
    std::vector<std::pair<int32_t, int32_t>> order;  // (mesh, old cell) in new order
    for (int L = 0; L <= depth; ++L) {
        for (size_t i = 0; i < n; ++i) {
            const HostPlan &h = *in[i];
            if (L > h.depth) continue;
            for (int32_t c = h.level_begin[L]; c < h.level_begin[L + 1]; ++c) {
                remap[i][c] = (int32_t)order.size();
                order.push_back({(int32_t)i, c});
            }
        }
        out.level_begin.push_back((int32_t)order.size());
    }
    out.cells.resize(order.size());
    for (size_t nc = 0; nc < order.size(); ++nc) {
        const size_t i = (size_t)order[nc].first;
        const HostPlan &h = *in[i];
        const Cell &C = h.cells[order[nc].second];
        Cell K = C;
        const double s = std::ldexp(1.0, -C.level);
        K.c[0] = ((double)C.ix + 0.5) * s;
        K.c[1] = ((double)C.iy + 0.5) * s;
        K.c[2] = ((double)C.iz + 0.5) * s;
        K.tbeg = (int32_t)(tet_off[i] + C.tbeg);
        K.tend = (int32_t)(tet_off[i] + C.tend);
        K.xbeg = (int32_t)(node_off[i] + C.xbeg);
        K.xend = (int32_t)(node_off[i] + C.xend);
        K.cbeg = C.nchild > 0 ? remap[i][C.cbeg] : (int32_t)out.cells.size();
        K.parent = C.parent >= 0 ? remap[i][C.parent] : -1;
        K.rsrc = C.rsrc / h.side;
        K.rtgt = C.rtgt / h.side;
        out.cells[nc] = K;
    }
    // children stay contiguous: a parent's children are consecutive cells of
    // one level of one mesh, which keep their order
    for (const Cell &K : out.cells)
        for (int32_t k = 1; k < K.nchild; ++k)
            if (out.cells[K.cbeg + k].parent != out.cells[K.cbeg].parent) throw PlanError{TFMM_ENOTSUP, "merge broke a sibling run"};
    // lists
    const int64_t nc = (int64_t)out.cells.size();
    std::map<std::array<int32_t, 4>, int32_t> kid;
    out.m2l_ptr.assign(nc + 1, 0);
    for (int64_t c = 0; c < nc; ++c) {
        const HostPlan &h = *in[order[c].first];
        const int32_t oc = order[c].second;
        out.m2l_ptr[c + 1] = out.m2l_ptr[c] + (h.m2l_ptr[oc + 1] - h.m2l_ptr[oc]);
    }
    out.m2l_src.resize((size_t)out.m2l_ptr[nc]);
    out.m2l_pair_key.resize((size_t)out.m2l_ptr[nc]);
    for (int64_t c = 0; c < nc; ++c) {
        const size_t i = (size_t)order[c].first;
        const HostPlan &h = *in[i];
        const int32_t oc = order[c].second;
        int32_t w = out.m2l_ptr[c];
        for (int32_t j = h.m2l_ptr[oc]; j < h.m2l_ptr[oc + 1]; ++j, ++w) {
            out.m2l_src[w] = remap[i][h.m2l_src[j]];
            const int32_t *kk = &h.m2l_keys[4 * (size_t)h.m2l_pair_key[j]];
            const std::array<int32_t, 4> key{kk[0], kk[1], kk[2], kk[3]};
            auto it = kid.find(key);
            if (it == kid.end()) {
                it = kid.emplace(key, (int32_t)(out.m2l_keys.size() / 4)).first;
                out.m2l_keys.insert(out.m2l_keys.end(), key.begin(), key.end());
            }
            out.m2l_pair_key[w] = it->second;
        }
    }
    for (size_t i = 0; i < n; ++i) {
        const HostPlan &h = *in[i];
        for (size_t k = 0; k < h.p2p_a.size(); ++k) {
            out.p2p_a.push_back(remap[i][h.p2p_a[k]]);
            out.p2p_b.push_back(remap[i][h.p2p_b[k]]);
        }
    }
}

void build_near_operator_layout(const HostPlan &hp, NearOpLayout &out)
{
    const int64_t C = (int64_t)hp.cells.size();
    std::vector<int32_t> cnt(C + 1, 0);
    for (int32_t a : hp.p2p_a) cnt[a + 1]++;
    for (int64_t c = 0; c < C; ++c) cnt[c + 1] += cnt[c];
    std::vector<int32_t> src(hp.p2p_b.size());
    {
        std::vector<int32_t> fillp(cnt.begin(), cnt.end() - 1);
        for (size_t i = 0; i < hp.p2p_a.size(); ++i) src[fillp[hp.p2p_a[i]]++] = hp.p2p_b[i];
    }
    out.leaf_off.assign(2 * (size_t)C, -1);
    out.leaf_nc.assign((size_t)C, 0);
    out.cols.clear();
    out.nvals = 0;
    out.nnz = 0;
    std::vector<int64_t> stamp((size_t)hp.n_nodes, -1);
    std::vector<int32_t> buf;
    for (int64_t a = 0; a < C; ++a) {
        const Cell &A = hp.cells[a];
        const int64_t nt = A.xend - A.xbeg;
        if (cnt[a + 1] == cnt[a] || nt == 0) continue;
        buf.clear();
        for (int32_t j = cnt[a]; j < cnt[a + 1]; ++j) {
            const Cell &Bc = hp.cells[src[j]];
            for (int32_t t = Bc.tbeg; t < Bc.tend; ++t)
                for (int c = 0; c < 4; ++c) {
                    const int32_t n = hp.tet_nodes[4 * (size_t)t + c];
                    if (stamp[n] != a) {
                        stamp[n] = a;
                        buf.push_back(n);
                    }
                }
        }
        if (buf.empty()) continue;
        std::sort(buf.begin(), buf.end());
        const int64_t nc = (int64_t)buf.size(), pad = (nc + 7) / 8 * 8;
        out.leaf_off[2 * a] = (int64_t)out.cols.size();
        out.leaf_off[2 * a + 1] = out.nvals;
        out.leaf_nc[a] = (int32_t)pad;
        out.cols.insert(out.cols.end(), buf.begin(), buf.end());
        out.cols.insert(out.cols.end(), (size_t)(pad - nc), buf.back());
        out.nvals += nt * 3 * pad;
        out.nnz += nt * nc;
    }
}

void build_near_topology(const HostPlan &hp, const std::vector<int32_t> &blk, NearTopo &out)
{
    static const int kEa[6] = {0, 0, 0, 1, 1, 2}, kEb[6] = {1, 2, 3, 2, 3, 3};
    static const int kFv[4][3] = {{1, 2, 3}, {0, 3, 2}, {0, 1, 3}, {0, 2, 1}};
    out = NearTopo{};
    out.inc.assign((size_t)hp.n_tets * 10, -1);
    const size_t nblk = blk.size() / 4;
    std::vector<int32_t> nodes, edges, faces;  // chunk: node ids, (a,b) id pairs, (p,q,r) id triples
    auto find = [](const std::vector<int32_t> &v, const int32_t *key, int w) -> int {
        for (size_t i = 0; i < v.size() / w; ++i) {
            bool eq = true;
            for (int k = 0; k < w; ++k) eq = eq && v[i * w + k] == key[k];
            if (eq) return (int)i;
        }
        return -1;
    };
    for (size_t b = 0; b < nblk; ++b) {
        const int32_t tb = blk[4 * b], te = blk[4 * b + 1];
        out.blk.push_back((int32_t)(out.ch_i.size() / 8));
        int32_t s = tb;
        while (s < te) {
            nodes.clear();
            edges.clear();
            faces.clear();
            int32_t t = s;
            for (; t < te && t - s < kTopoTets; ++t) {
                const int32_t *v = &hp.tet_nodes[4 * (size_t)t];
                // entities this tet would add
                std::vector<int32_t> nn, ne, nf;
                for (int c = 0; c < 4; ++c)
                    if (find(nodes, &v[c], 1) < 0 && find(nn, &v[c], 1) < 0) nn.push_back(v[c]);
                for (int e = 0; e < 6; ++e) {
                    const int32_t key[2] = {std::min(v[kEa[e]], v[kEb[e]]), std::max(v[kEa[e]], v[kEb[e]])};
                    if (find(edges, key, 2) < 0 && find(ne, key, 2) < 0) ne.insert(ne.end(), key, key + 2);
                }
                for (int k = 0; k < 4; ++k) {
                    int32_t key[3] = {v[kFv[k][0]], v[kFv[k][1]], v[kFv[k][2]]};
                    std::sort(key, key + 3);
                    if (find(faces, key, 3) < 0 && find(nf, key, 3) < 0) nf.insert(nf.end(), key, key + 3);
                }
                if (nodes.size() + nn.size() > (size_t)kTopoNodes || (edges.size() + ne.size()) / 2 > (size_t)kTopoEdges ||
                    (faces.size() + nf.size()) / 3 > (size_t)kTopoFaces)
                    break;
                nodes.insert(nodes.end(), nn.begin(), nn.end());
                edges.insert(edges.end(), ne.begin(), ne.end());
                faces.insert(faces.end(), nf.begin(), nf.end());
                for (int e = 0; e < 6; ++e) {
                    const int32_t key[2] = {std::min(v[kEa[e]], v[kEb[e]]), std::max(v[kEa[e]], v[kEb[e]])};
                    out.inc[10 * (size_t)t + e] = find(edges, key, 2);
                }
                for (int k = 0; k < 4; ++k) {
                    int32_t key[3] = {v[kFv[k][0]], v[kFv[k][1]], v[kFv[k][2]]};
                    std::sort(key, key + 3);
                    out.inc[10 * (size_t)t + 6 + k] = find(faces, key, 3);
                }
            }
            // chunk record
            const int32_t noff = (int32_t)(out.nd_w.size() / 3), eoff = (int32_t)out.ed_il.size(),
                          foff = (int32_t)(out.fc_n.size() / 3);
            double c[3] = {0.0, 0.0, 0.0};
            for (int32_t id : nodes)
                for (int k = 0; k < 3; ++k) c[k] += hp.nodes[3 * (size_t)id + k];
            for (int k = 0; k < 3; ++k) c[k] /= (double)nodes.size();
            auto local = [&](int32_t id) { return find(nodes, &id, 1); };
            auto pos = [&](int32_t id, int k) { return hp.nodes[3 * (size_t)id + k] - c[k]; };
            for (int32_t id : nodes)
                for (int k = 0; k < 3; ++k) out.nd_w.push_back(pos(id, k));
            for (size_t e = 0; e < edges.size() / 2; ++e) {
                const int32_t a = edges[2 * e], bb = edges[2 * e + 1];
                out.ed_ab.push_back(local(a));
                out.ed_ab.push_back(local(bb));
                double d2 = 0.0;
                for (int k = 0; k < 3; ++k) {
                    const double dk = pos(bb, k) - pos(a, k);
                    d2 += dk * dk;
                }
                out.ed_il.push_back(1.0 / std::sqrt(d2));
            }
            for (size_t f = 0; f < faces.size() / 3; ++f) {
                const int32_t pp = faces[3 * f], qq = faces[3 * f + 1], rr = faces[3 * f + 2];
                out.fc_pqr.push_back(local(pp));
                out.fc_pqr.push_back(local(qq));
                out.fc_pqr.push_back(local(rr));
                double u[3], w[3];
                for (int k = 0; k < 3; ++k) {
                    u[k] = pos(qq, k) - pos(pp, k);
                    w[k] = pos(rr, k) - pos(pp, k);
                }
                const double n[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
                const double il = 1.0 / std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
                for (int k = 0; k < 3; ++k) out.fc_n.push_back(n[k] * il);
                out.fc_a2.push_back(1.0 / il);
            }
            const int32_t rec[8] = {s, t - s, noff, (int32_t)nodes.size(), eoff, (int32_t)(edges.size() / 2), foff,
                                    (int32_t)(faces.size() / 3)};
            out.ch_i.insert(out.ch_i.end(), rec, rec + 8);
            out.ch_c.insert(out.ch_c.end(), c, c + 3);
            s = t;
        }
        out.blk.push_back((int32_t)(out.ch_i.size() / 8));
        out.blk.push_back(blk[4 * b + 2]);
        out.blk.push_back(blk[4 * b + 3]);
    }
}

}  // namespace tfmm
