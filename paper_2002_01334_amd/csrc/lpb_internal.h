// lpb_internal.h -- plan (trees, lists, operator descriptors) shared by the
// host plan builder, the operator generator and the evaluation kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/lpb.h"
#include "lpb_math.h"

namespace lpb {

constexpr int kMaxDepth = 12;   // deepest tree level
constexpr int kCellBits = 16;   // fine cell bits per axis
constexpr int kTileMinLevel = 4;  // free-space levels kTileMinLevel..kTileMaxLevel use the tiled MFMA M2L
constexpr int kTileMaxLevel = 8;  // (coarser grids are mostly boundary: their pairs go to the batched kernel)
constexpr int kTilePB = 4;        // parents per axis of an M2L tile (4^3 parents -> 64 target boxes)
constexpr int kTileMinBoxes = 16; // tiles with fewer target boxes give their pairs to the batched list
constexpr int kVOffsets = 189;    // V-list offsets of one child octant
// Tiled levels store one operator per offset with non-negative components;
// the offset (sx dx, sy dy, sz dz) uses it between sign flips D = diag(+-1)
// of both the source and the result (reflection bits: 1 x, 2 y, 4 z).
constexpr int kReflShift = 28;
// Untiled V-list pairs share operators the same way per pair: free-space
// pairs by reflection (code 0..7, A_d = D A_|d| D) and reaction pairs by
// rotation about z (codes kXfRotate + dir): the reaction translation depends
// on the azimuth phi of c_t - c_s only through e^{i(mu - m) phi}, so
// T(phi) = diag(e^{-i m phi}) T(0) diag(e^{i mu phi}) and one operator per
// (level, rho, z_t, z_s) serves every direction.  A V-list source box sits
// (dx, dy) cells from its target box with |dx|, |dy| <= 3, so phi =
// atan2(-dy, -dx) takes one of kXfDirs values, dir = (dx + 3) 7 + (dy + 3),
// and cos / sin (m phi) come from a table (EvalArgs::rot_tab).
constexpr int kXfRotate = 8;
constexpr int kXfDirs = 49;
// The 189 offsets of a child octant form 56 orbits under those reflections
// (canonical offset (|dx|,|dy|,|dz|)).  Per axis an orbit has both signs
// ("both" axes, 1 or 2 away) or one (0, or 3 on the side the octant allows).
// orb_tab holds per octant and orbit kOrbTab entries:
//   [0]      nb | both << 4 | minus << 7: nb the number of both-axes, both
//            their mask, minus the mask of the one-sign axes whose sign is
//            negative;
//   [1..8]   the 2^nb members in compact order j (member reflection code
//            deposit(j, both) | minus), as offsets in the 13^3 local source
//            grid of a tile, ((dx+3) 13 + dy+3) 13 + dz+3;
//   [9..16]  for the transform outputs (j + (t << nb)): class g << 12 with the
//            sign (-1)^|g & minus| in bit 31, g = deposit(j, both) |
//            deposit(t, one-sign axes);
//   [17]     the canonical offset code ((a+3) 7 + b+3) 7 + c+3.
// The table lists the orbits of an octant in 8 groups of kOrbGroup, one per
// both-axes mask (which does not depend on the octant), in the order
// kOrbGroupMask: member counts 8, 4, 4, 4, 2, 2, 2, 1 never increase.
constexpr int kOrbits = 56;
constexpr int kOrbTab = 18;
constexpr int kOrbGroup = 7;
constexpr int kOrbGroupMask[8] = {7, 6, 5, 3, 4, 2, 1, 0};
constexpr int kOrbGrid = 13;    // local source grid of a tile (4 parents x 2 + 6 halo per axis)
constexpr int kOrbitMinP = 5;   // below, class padding outweighs the saving
constexpr int kOrbitMaxP = 15;

enum OpType { OP_M2M = 0, OP_L2L = 1, OP_M2L_FREE = 2, OP_M2L_REACT = 3 };

// One FMM of the plan: a free-space Yukawa FMM of layer l (kind 0) or the
// reaction component (l, lp, a, b) over equivalent polarization sources
// (kind 1).  All geometry below is in the FMM's canonical frame: origin at
// the root centre, z flipped (flip = -1) for a = 2 so that targets always lie
// above the interface (canonical z > 0) and images below.
struct FmmDesc {
    int sys, kind, l, lp, a, b;
    double cx, cy, cz, R;     // root centre (original frame) and half side
    int flip;                 // +1 or -1
    int H;                    // depth
    double lam_s, lam_t;      // source-side and target-side lambda
    double far_factor;        // multiplies the far field (free space: lam/(2 pi^2 eps))
    double eps_t;             // eps of the target layer (free-space near field)
    int slot;                 // output slot of this FMM's targets
    int me_off[kMaxDepth + 1];   // first ME box of each level (global index), -1 below level 2
    int le_off[kMaxDepth + 1];
    int nsrc, ntgt;
    int layers_id;            // which layered medium (system) for sigma
    int src_tree, tgt_tree;   // the (possibly shared) trees of its sources and targets
};

// A point set on its uniform octree: the sources of an FMM (ME boxes) or its
// targets (LE boxes).  Reaction components share the trees of their
// (layer, side) sets; the representative FMM lends lambda and root.
struct TreeDesc {
    int target;   // 0 source tree, 1 target tree
    int rep;      // representative FMM
    int H;
    int leaf0, nleaf;
};

// Device-resident description of one medium for the reaction densities.
struct Medium {
    int L;
    double eps[LPB_MAXL + 1];
    double lam[LPB_MAXL + 1];
    double d[LPB_MAXL];
};

// Per-FMM record used by the kernels (device).
struct FmmDev {
    int kind;
    int H;
    int flip;
    int medium;
    int l, lp, a, b;
    double R;
    double lam_s, lam_t;
    double far_factor, eps_t;
    int me_off[kMaxDepth + 1];
    int le_off[kMaxDepth + 1];
};

// Operator descriptor (generation input).
struct OpDesc {
    int type;        // OpType
    int fmm;
    int level;       // level of the box the operator writes (M2M: parent level; L2L, M2L: target level)
    int rkey;        // reaction geometry key (OP_M2L_REACT) or -1
    double bx, by, bz;  // free ops: translation vector b of the addition theorem (canonical frame)
    double phi;      // reaction: azimuth of (target centre - source centre)
};

// Reaction geometry key: phi-independent part of a reaction M2L operator.
struct RKey {
    int fmm, level;
    double rho, zt, zs;   // canonical: zt > 0 (target centre height), zs < 0 (source centre)
    double S;             // box side (scaling length of the paper's scaled integrals)
};

// Reaction point operator (adaptive trees, Sec. 3.5 closing remarks): for
// kind 0 (M2P) the row that evaluates the scaled ME of a source box at one
// target point, for kind 1 (P2L) the scaled LE of a target box due to one
// unit source point; K doubles at `out`.  pt: the point (index into the
// target or source arrays), leaf: its leaf; (bx, by, bz): the box centre and
// h its side, canonical frame.
struct PointOp {
    int kind, fmm, pt, leaf;
    double bx, by, bz, h;
    int64_t out;
};

// Tiled free-space M2L: one record per (free FMM, level) with dense box grids,
// and tiles of 64 target boxes sharing a child octant (so that all of them
// have the same 189 V-list offsets and operators).
struct TileFL {
    int fmm, level, nside;
    int grid_off;     // into grid_me / grid_le (nside^3 entries each)
    int optab_off;    // into optab (343 entries: offset code -> operator | reflection << kReflShift)
};
struct Tile {
    int fl, octant, px0, py0, pz0;
};

// Host-side plan (built by build_plan, uploaded by the context).
struct Plan {
    int p = 10, K = 121, leaf_cap = 50;
    int nsys = 0;
    std::vector<int64_t> sys_charge_off;   // nsys + 1
    std::vector<Medium> media;             // per system
    std::vector<FmmDesc> fmm;
    std::vector<TreeDesc> trees;
    int nslots = 1;                        // output slots per charge
    int64_t ncharges = 0;
    int max_depth = 0;
    // points (sources and targets sorted by FMM, then leaf): they stay on the
    // device; the plan lists the point sets of the builder (PointBuilder
    // handles) in tree order, each target set with its output slot
    int64_t n_spts = 0, n_tpts = 0;
    std::vector<int> s_sets, t_sets, t_set_slot;
    // leaves
    std::vector<int> sl_start, sl_me, sl_fmm, sl_tree;    // source leaves (sl_start has n+1); sl_fmm: representative
    std::vector<int> tl_start, tl_le, tl_fmm, tl_tree;    // target leaves
    std::vector<double> sl_h, tl_h;                       // leaf box side
    std::vector<double> sl_ctr, tl_ctr;                   // leaf centres (canonical local frame), 3 per leaf
    std::vector<uint64_t> sl_cell, tl_cell;               // leaf cells (canonical, diagnostics)
    std::vector<int> sl_lv, tl_lv;                        // leaf levels (all H on uniform trees)
    // boxes
    int n_me = 0, n_le = 0;
    // M2L: CSR by target LE box
    std::vector<int> m2l_ptr, m2l_src, m2l_op;   // m2l_ptr has n_le+1
    // per pair: how the pair's operator relates to the stored one (see kXfRotate)
    std::vector<int> m2l_xc;
    // batched dense translations on the matrix cores: work item w has terms
    // [bw_term_ptr[w], bw_term_ptr[w+1]), term t = operator bw_op[t] and 64
    // source rows bw_src[64 t + j]; 64 destination rows bw_dst[64 w + j] (-1: none)
    std::vector<int> bw_term_ptr, bw_op, bw_src, bw_dst;
    std::vector<int> bw_xc;      // per column: -1 none, 0..7 reflection code, kXfRotate + dir rotation
    std::vector<int> bm2m_lv, bl2l_lv;   // work items of M2M (parent level) / L2L (child level) l: [v[l], v[l+1])
    int bm2l_w0 = 0, bm2l_w1 = 0;        // V-list pairs outside the tiled levels, grouped by operator;
                                         // destination = the pair's position in m2l_src (scratch row)
    // near field: CSR by target leaf over free-space source leaves, and over
    // (reaction FMM, source leaf) pairs
    std::vector<int> p2p_ptr, p2p_src;
    std::vector<int> rp_ptr, rp_fmm, rp_src;
    int64_t n_p2p_pairs = 0, n_react_p2p_pairs = 0, n_m2l_pairs = 0, n_m2l_tile_pairs = 0;
    // adaptive trees: W-list (M2P) CSR by target leaf, entries (FMM, source
    // ME box, its level, its centre in the canonical frame, first point
    // operator or -1); X-list (P2L) per target LE box (w_* analogues x_box_*)
    // with entries (FMM, source leaf, first point operator or -1).  Reaction
    // entries evaluate precomputed point operators (one K-vector per target
    // point of the leaf, or per source point of the leaf); free-space entries
    // the closed forms.
    int adaptive = 0;   // 0 uniform, 1 adaptive (with the reaction sets' separation rule), 2 occupancy only
    std::vector<int> w_ptr, w_fmm, w_me, w_lv;
    std::vector<double> w_ctr;
    std::vector<int64_t> w_vec;
    std::vector<int> x_box_le, x_box_lv, x_box_ptr;
    std::vector<double> x_box_ctr;
    std::vector<int> x_fmm, x_sl;
    std::vector<int64_t> x_vec;
    std::vector<PointOp> pt_ops;   // reaction point operators to generate
    int64_t n_w_pairs = 0, n_x_pairs = 0, n_w_points = 0, n_x_points = 0;
    // operators
    std::vector<OpDesc> ops;
    std::vector<RKey> rkeys;
    // tiled free-space M2L
    std::vector<TileFL> tfl;
    std::vector<Tile> tiles;
    std::vector<int> grid_me, grid_le, optab;
    std::vector<int> oct_codes;    // 8 x 189 offset codes ((dx+3)*7+(dy+3))*7+(dz+3)
    std::vector<int> orb_tab;      // 8 x kOrbits x kOrbTab (see kOrbits)
    std::vector<int> orb_ops;      // canonical operators of the tiled levels
    std::vector<int> orb_index;    // op -> position in orb_ops, -1 if none
    std::vector<int> swz_ops;      // operators stored in the MFMA operand layout (all of them)
    std::vector<int> swz_index;    // op -> position in swz_ops
};

// Canonical frame of a point set: w = (x - ax, y - ay, wz) with wz = z - az
// for a free-space set (mode 0); for a reaction set (mode 1) t = z - az on
// side 1 (az = d_l) or az - z on side 2 (az = d_{l-1}), and wz = t for its
// targets, -t for its images.
struct SetFrame {
    int mode, side, target;
    double ax, ay, az;
};

// The per-point part of the plan builder: canonical coordinates, fine cells
// and keys, the sort, the leaves and each point's offset from its leaf
// centre.  The points stay with the builder; the plan gets counts, leaf keys
// and leaf starts.
class PointBuilder {
public:
    virtual ~PointBuilder() = default;
    // Sort the points `members` (indices into system sys, increasing; global
    // charge index coff + member) by the Morton key of their fine cell in
    // frame F with root half side R, equal keys in charge order; counts[l] =
    // distinct level-l cells, l = 0..kMaxDepth.  Returns a handle >= 0, or -1
    // with msg set.
    virtual int keys(int sys, int64_t coff, const std::vector<int>& members, const SetFrame& F, double R,
                     int counts[kMaxDepth + 1], std::string& msg) = 0;
    // The set's leaves at depth H (leaf_key: level-H Morton keys in order,
    // leaf_start: first point of each leaf); computes the points' offsets from
    // their leaf centres.  False with msg set on failure.
    virtual bool leaves(int handle, int H, std::vector<uint64_t>& leaf_key, std::vector<int>& leaf_start,
                        std::string& msg) = 0;
    // Adaptive leaves: boxes divided while they hold more than cap points,
    // and with sep (a reaction set) while they are wider than the distance
    // of their nearest point from the interface plane, up to 3 levels below
    // the occupancy rule's (all down to kMaxDepth; distances and widths in
    // fine cells, the plane between z cells 32767 and 32768); leaf_key at
    // each leaf's own level leaf_lv, in Morton order, leaf_start its first
    // point; computes the points' offsets from their leaf centres.  False
    // with msg set on failure.
    virtual bool leaves_adaptive(int handle, int cap, bool sep, std::vector<uint64_t>& leaf_key,
                                 std::vector<int>& leaf_lv, std::vector<int>& leaf_start, std::string& msg) = 0;
    // lpb_status of the last failure (LPB_ENOMEM or LPB_EDEVICE)
    virtual int failure() const = 0;
};

// Build the plan for all systems (boxes, lists and operators on the host,
// points through `pb`).  Returns an error message or "".
std::string build_plan(Plan& P, const std::vector<Medium>& media, const std::vector<std::vector<double>>& xs,
                       const std::vector<std::vector<double>>& ys, const std::vector<std::vector<double>>& zs,
                       double iface_tol, PointBuilder& pb, int* status);

// the low 16 bits of v spread to every third bit (a level-l Morton key is
// spread3(ix) << 2 | spread3(iy) << 1 | spread3(iz))
inline uint64_t morton_spread3(uint32_t v)
{
    uint64_t x = v & 0xffffu;
    x = (x | (x << 16)) & 0x0000ff0000ffull;
    x = (x | (x << 8)) & 0x00f00f00f00full;
    x = (x | (x << 4)) & 0x0c30c30c30c3ull;
    x = (x | (x << 2)) & 0x249249249249ull;
    return x;
}

// level-l cell coordinates of a level-l Morton key (bits x, y, z interleaved)
inline uint32_t morton_compact3(uint64_t x)
{
    x &= 0x249249249249ull;
    x = (x | (x >> 2)) & 0x0c30c30c30c3ull;
    x = (x | (x >> 4)) & 0x00f00f00f00full;
    x = (x | (x >> 8)) & 0x0000ff0000ffull;
    x = (x | (x >> 16)) & 0xffffull;
    return (uint32_t)x;
}

// Layer of height z: number of interfaces above z.
inline int layer_of(const Medium& m, double z)
{
    int l = 0;
    for (int k = 0; k < m.L; ++k)
        if (m.d[k] > z) l = k + 1;
    return l;
}

double host_gaunt(int n1, int m1, int n2, int m2, int n3, int m3);

// Morton key at level H of a leaf cell (cellkey packing), with the z cell
// mirrored when flip < 0 (original orientation of an a = 2 component).
uint64_t leaf_key(uint64_t lcell, int H, int flip);

}  // namespace lpb
