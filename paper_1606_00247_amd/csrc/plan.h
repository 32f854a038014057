// Host-side plan of the tetrahedral FMM: validated and oriented mesh, octree
// over tets and targets, cell radii and the interaction lists of the dual tree
// traversal.  Pure C++ (no HIP); compiled without floating-point contraction
// so that every discrete decision (octant keys, radii, the acceptance test) is
// reproducible bit for bit.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace tfmm {

struct Cell {
    int32_t level;
    int32_t ix, iy, iz;
    double c[3];           // geometric centre of the cube
    int32_t tbeg, tend;    // tets [tbeg, tend) in sorted order
    int32_t xbeg, xend;    // targets [xbeg, xend) in sorted order
    int32_t cbeg, nchild;  // children are cells [cbeg, cbeg + nchild)
    int32_t parent;        // -1 for the root
    double rsrc, rtgt;     // acceptance radii (Sec. 3.2)
};

struct HostPlan {
    // parameters
    int p = 0, leaf = 0;
    double theta = 0.0;
    int64_t n_nodes = 0, n_tets = 0, n_targets = 0;
    bool targets_are_nodes = true;
    bool points = false;  // sources are point dipoles at the nodes (see build_host_plan)

    // bounding cube
    double origin[3] = {0, 0, 0};
    double side = 0.0;

    // mesh (input order)
    std::vector<double> nodes;  // [n_nodes][3]

    // tets in octree order, corners oriented to positive volume
    std::vector<int32_t> tet_perm;  // sorted -> input tet index
    std::vector<int32_t> tet_nodes; // [n_tets][4] node indices

    // targets in octree order
    std::vector<int32_t> tgt_perm;  // sorted -> input target index
    std::vector<double> tgt_xyz;    // [n_targets][3] sorted

    // tree: cells grouped by level, children of one parent contiguous
    std::vector<Cell> cells;
    std::vector<int32_t> level_begin;  // cells of level L are [level_begin[L], level_begin[L+1])
    int depth = 0;

    // interaction lists
    std::vector<int32_t> m2l_ptr, m2l_src;  // CSR by target cell
    std::vector<int32_t> p2p_a, p2p_b;      // P2P leaf pairs (target, source)
    int64_t n_p2p_pairs = 0;                // sum of ntargets(A) * ntets(B)

    // M2L translation keys: key = (dlevel, kx, ky, kz), dlevel = level(B) -
    // level(A), k = (c_A - c_B) in units of half the smaller cube side (exact
    // integers); one key id per M2L pair (same order as m2l_src)
    std::vector<int32_t> m2l_keys;      // [nkeys][4]
    std::vector<int32_t> m2l_pair_key;  // [n_m2l]

    double setup_seconds = 0.0;
};

// M2L grouped for matrix cores: target cells in tiles of `tpt` cells of one
// level; per tile a list of entries, one per distinct key used by its cells
// (sorted by level difference, then key), with the source cell of each tile
// slot (-1: none).  A tile's entries are cut into work items of at most
// max_ent entries (each adds its part to the tiles' local expansions), and
// the work items are ordered for dispatch over the XCDs: each XCD takes a
// spatially contiguous share of every level, longest items first (empty
// items, tile_rng {0, 0}, pad the XCDs with fewer).
constexpr int kM2LXcds = 8;
struct M2LTiles {
    int tpt = 0;
    std::vector<int32_t> tile_tgt;  // [nitems][tpt] target cells (-1: empty slot)
    std::vector<int32_t> tile_rng;  // [nitems][2] entry range [begin, end)
    std::vector<int32_t> ent_key;   // [nent]
    std::vector<int32_t> ent_src;   // [nent][tpt]
};

// M2L grouped by key inside blocks of target cells (the form for fewer than
// 16 fields).  A block holds up to nb target cells of one level, consecutive
// in Morton order; its translations are sorted by key, and the pairs of one
// key are packed into groups of tpg = 16 / fpt (target slot, source cell)
// pairs, so that every matrix-core column of a group carries a translation
// except in the last group of each key.  A work item is a run of at most
// max_grp groups of one block; items are ordered for the XCDs as the tiles.
struct M2LPacks {
    int nb = 0, tpg = 0;
    std::vector<int32_t> blk_cells;  // [nblk][nb] target cells (-1: empty slot)
    std::vector<int32_t> item;       // [nitems][3] block, group begin, group end
    std::vector<int32_t> grp_key;    // [ngrp]
    std::vector<int32_t> grp_src;    // [ngrp][tpg] source cell (-1: empty)
    std::vector<uint8_t> grp_slot;   // [ngrp][tpg] target slot in the block
};
void build_m2l_packs(const HostPlan &hp, int nb, int tpg, int max_grp, M2LPacks &out, int only_level = -1);

// Mesh entities of the near-field source blocks.  Each P2P block (<= 64 tets
// of one leaf, [tbeg, tend) in octree order) is cut into chunks of at most
// kTopoTets tets with at most kTopoNodes distinct nodes, kTopoEdges edges and
// kTopoFaces faces; per chunk the distinct nodes (positions relative to the
// chunk's node centroid), edges (canonical direction: lower node id first,
// inverse length) and faces (nodes in increasing id order, unit normal of
// that order), and per tet the chunk-local indices of its 6 edges (corner
// pairs (0,1),(0,2),(0,3),(1,2),(1,3),(2,3)) and 4 faces (face k opposite
// corner k).
constexpr int kTopoTets = 16, kTopoNodes = 16, kTopoEdges = 48, kTopoFaces = 40;
struct NearTopo {
    std::vector<int32_t> blk;     // [nblk][4]: chunk begin, chunk end, target begin, target end
    std::vector<int32_t> ch_i;    // [nch][8]: tbeg, ntets, node off, nodes, edge off, edges, face off, faces
    std::vector<double> ch_c;     // [nch][3] node centroid
    std::vector<double> nd_w;     // [nodes][3] position - centroid
    std::vector<int32_t> ed_ab;   // [edges][2] chunk-local nodes
    std::vector<double> ed_il;    // [edges] 1 / length
    std::vector<int32_t> fc_pqr;  // [faces][3] chunk-local nodes
    std::vector<double> fc_n;     // [faces][3] unit normal of (q - p) x (r - p)
    std::vector<double> fc_a2;    // [faces] |(q - p) x (r - p)| (twice the area)
    std::vector<int32_t> inc;     // [T][10] per tet: 6 edge, 4 face chunk-local indices
};

// Stored near-field operator (the node-to-node coefficients of the direct
// part, Sec. 2.1, assembled once per mesh).  With the tets of the P2P source
// leaves of a target leaf A written out by their nodes, the near potential at
// a target x of A is sum_j C_xj . M_j over the distinct nodes j of those tets:
// per target leaf one sorted column list (padded to a multiple of 8 by
// repeating its last node) and one dense coefficient block [nt(A)][3][ncols].
struct NearOpLayout {
    std::vector<int64_t> leaf_off;  // [C][2]: column offset, value offset (-1: no block)
    std::vector<int32_t> leaf_nc;   // [C] padded column count
    std::vector<int32_t> cols;      // node ids, per leaf sorted
    int64_t nvals = 0;              // doubles in all blocks
    int64_t nnz = 0;                // (target, node) pairs before padding
};
void build_near_operator_layout(const HostPlan &hp, NearOpLayout &out);

// Builds the chunks of the P2P blocks blk ([nblk][4]: tbeg, tend, ibeg, iend).
void build_near_topology(const HostPlan &hp, const std::vector<int32_t> &blk, NearTopo &out);

// Error raised by the plan builder: code is one of the TFMM_E* values.
struct PlanError {
    int code;
    std::string msg;
};

// Groups the M2L pairs of a built plan into target tiles of tpt cells and
// work items of at most max_ent entries (only target cells of level
// only_level when it is >= 0).
void build_m2l_tiles(const HostPlan &hp, int tpt, int max_ent, M2LTiles &out, int only_level = -1);

// One plan over several meshes (a ragged batch): the plans `in` (same p,
// leaf and theta, tet sources, targets = nodes) are normalised to their own
// root cube (origin 0, side 1: coordinates x' = (x - origin) / side) and
// concatenated: nodes, tets and targets in mesh order, cells grouped by
// level (mesh by mesh within a level, each mesh's order kept), lists with
// their cell indices remapped, keys unified.  Trees, radii and lists are
// those of the meshes, so no mesh interacts with another.  The potential of
// a mesh in its normalised frame is its true potential divided by its root
// side (u scales with length at fixed M): scale[i] = side_i; node_off[i] is
// the first node (and target) of mesh i (node_off.back() = total).
void merge_host_plans(const std::vector<const HostPlan *> &in, HostPlan &out, std::vector<double> &scale,
                      std::vector<int64_t> &node_off);

// Builds the plan.  Throws PlanError on invalid input.  With points = true
// the sources are the n_nodes points `nodes` (tets is ignored).
void build_host_plan(HostPlan &hp, const double *nodes, int64_t n_nodes, const int32_t *tets, int64_t n_tets,
                     const double *targets, int64_t n_targets, int p, int leaf, double theta, bool points = false);

}  // namespace tfmm
