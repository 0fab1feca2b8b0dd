// lpb_plan.cpp -- host construction of the FMM plan: layers of the charges,
// equivalent polarization coordinates, one uniform octree per FMM, the
// interaction lists and the operator descriptors.
//
// Tree rule (identical in meaning to the oracle's, written independently):
//   free space: root cube = centre of the bounding box of the layer's
//     charges, half side = half the largest extent; depth H = smallest l
//     (<= 12) with N <= cap * (non-empty boxes at l).
//   reaction components: one grid per medium.  In a component's frame
//     (interface at z = 0, targets above it, mirrored for a = 2) targets sit
//     at +tau and images at -tau (distance to an interface of their own
//     layer).  Root: centre x, y of the bounding box of all charges, z on
//     the interface (Sec. 3.5: the largest box is halved by it), half side =
//     max of the half x, y extents and every tau; depth = the largest of the
//     per-set rule over all (layer, side) sets, as images and as targets,
//     raised (by at most 3 levels) until the box side is <= the smallest tau.
//   fine cell per axis: floor((w + R) / (2R) * 65536) clamped to [0, 65535]
//     with w the canonical coordinate relative to the root centre; the
//     level-l cell is the fine cell >> (16 - l).
//   V-list (levels >= 2): source boxes that are children of the neighbours
//     of the target's parent and not adjacent to the target; U-list at level
//     H: the target's neighbours and itself.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <functional>
#include <unordered_map>

#include "lpb_internal.h"

namespace lpb {

namespace {

// Morton key of a level-l cell: bits interleaved x, y, z from the top level down.
uint64_t morton(uint32_t ix, uint32_t iy, uint32_t iz, int l)
{
    uint64_t k = 0;
    for (int bit = l - 1; bit >= 0; --bit)
        k = (k << 3) | ((uint64_t)((ix >> bit) & 1u) << 2) | ((uint64_t)((iy >> bit) & 1u) << 1) |
            (uint64_t)((iz >> bit) & 1u);
    return k;
}

inline uint64_t cellkey(int ix, int iy, int iz)
{
    return ((uint64_t)(uint32_t)ix << 42) | ((uint64_t)(uint32_t)iy << 21) | (uint64_t)(uint32_t)iz;
}

struct BoxSet {
    // level-l boxes of one point set: canonical cell coords sorted by Morton key
    std::vector<uint64_t> mkey;
    std::vector<int> ix, iy, iz;
    // cell -> position: a dense grid while it has at most kDenseRatio cells
    // per box (and at most kDenseSide^3), else a binary search of the keys
    static constexpr int kDenseSide = 128;
    static constexpr size_t kDenseRatio = 64;
    int nside = 0;
    bool use_dense = false;
    std::vector<int> dense;
    void init(int lv, size_t nbox)
    {
        nside = 1 << lv;
        const size_t cells = (size_t)nside * nside * nside;
        use_dense = nside <= kDenseSide && cells <= std::max<size_t>(4096, kDenseRatio * nbox);
        if (use_dense) dense.assign(cells, -1);
    }
    void insert(int a, int b, int c, int pos)
    {
        if (use_dense) dense[((size_t)a * nside + b) * nside + c] = pos;
    }
    // position of cell (a, b, c), -1 if empty or outside the grid
    int find(int a, int b, int c) const
    {
        if (a < 0 || b < 0 || c < 0 || a >= nside || b >= nside || c >= nside) return -1;
        if (use_dense) return dense[((size_t)a * nside + b) * nside + c];
        const uint64_t k = (morton_spread3((uint32_t)a) << 2) | (morton_spread3((uint32_t)b) << 1) | morton_spread3((uint32_t)c);
        auto it = std::lower_bound(mkey.begin(), mkey.end(), k);
        return (it != mkey.end() && *it == k) ? (int)(it - mkey.begin()) : -1;
    }
};

// One point set on its uniform octree, as built into the plan.
struct TreeB {
    std::vector<BoxSet> B;       // levels 0..H
    int off[kMaxDepth + 1];      // global ME (source tree) or LE (target tree) index of each level, -1 below 2
    int leaf0 = 0, nleaf = 0;    // its leaves in sl_* (source) or tl_* (target)
    int id = -1;                 // index into Plan::trees
};

// One batched work item (64 columns).
struct BWork {
    std::vector<int> op;    // per term
    std::vector<int> src;   // 64 per term
    std::array<int, 64> dst;
    std::array<int, 64> xc;      // per column transform code (-1 none)
    BWork() { xc.fill(-1); }
};

// Staging shared by the tree and list builders.
struct Staging {
    std::vector<std::vector<BWork>> bm2m{(size_t)kMaxDepth + 1}, bl2l{(size_t)kMaxDepth + 1};
    struct M2LPair { int le, src, op, xc; };
    std::vector<M2LPair> m2l_pairs;                             // untiled V-list pairs in list order (grouped by LE box at the end)
    // U-list entries in the order they are found: (target leaf, source leaf)
    // for free space, (target leaf, reaction FMM, source leaf) for reactions;
    // grouped by target leaf (stable) at the end
    std::vector<std::array<int, 2>> p2p_pairs;
    std::vector<std::array<int, 3>> rp_pairs;
    // adaptive trees: W-list (target leaf, FMM, source ME box, its level,
    // centre) and X-list (target LE box, its level, centre, FMM, source leaf)
    struct WPair { int tl, fmm, me, lv; double c[3]; };
    struct XPair { int le, lv; double c[3]; int fmm, sl; };
    std::vector<WPair> w_pairs;
    std::vector<XPair> x_pairs;
};

// A point set after the builder's sort: its handle, size and leaves.
struct PtsInfo {
    int handle = -1, n = 0;
    int counts[kMaxDepth + 1] = {};
    std::vector<uint64_t> lkey;   // Morton key of each leaf at its level (H, or llv on adaptive trees)
    std::vector<int> lstart;      // first point of each leaf
    std::vector<int> llv;         // adaptive trees: level of each leaf (empty: all at H)
    int leaf_level(size_t k, int H) const { return llv.empty() ? H : llv[k]; }
    int max_level() const
    {
        int m = 0;
        for (int v : llv) m = std::max(m, v);
        return m;
    }
};

// smallest level (<= kMaxDepth) at which N <= cap * (non-empty boxes)
inline int depth_rule(const PtsInfo& V, int cap)
{
    for (int lv = 0; lv < kMaxDepth; ++lv)
        if ((int64_t)V.n <= (int64_t)cap * V.counts[lv]) return lv;
    return kMaxDepth;
}

// Add one tree (boxes, leaves, points, and its M2M or L2L operators and lists)
// to the plan.  rep: the FMM whose lambda and root the tree's operators use.
void add_tree(Plan& P, Staging& S, const PtsInfo& V, int H, double R, bool target, int rep, int slot, TreeB& T)
{
    // the level-l boxes are the distinct level-l prefixes of the keys of the
    // leaves at level l or deeper, in key order
    const size_t nl = V.lkey.size();
    T.B.assign(H + 1, BoxSet{});
    for (int lv = 0; lv <= H; ++lv) {
        BoxSet& bs = T.B[lv];
        auto prefix = [&](size_t i, uint64_t& k) {
            const int L = V.leaf_level(i, H);
            if (L < lv) return false;
            k = V.lkey[i] >> (3 * (L - lv));
            return true;
        };
        size_t nb = 0;
        {
            bool have = false;
            uint64_t prev = 0, k;
            for (size_t i = 0; i < nl; ++i)
                if (prefix(i, k)) {
                    nb += !have || k != prev;
                    have = true;
                    prev = k;
                }
        }
        bs.init(lv, nb);
        bool have = false;
        uint64_t prev = 0;
        for (size_t i = 0; i < nl; ++i) {
            uint64_t k;
            if (!prefix(i, k)) continue;
            if (have && k == prev) continue;
            have = true;
            prev = k;
            const int a = (int)morton_compact3(k >> 2), b = (int)morton_compact3(k >> 1), c = (int)morton_compact3(k);
            bs.insert(a, b, c, (int)bs.mkey.size());
            bs.mkey.push_back(k);
            bs.ix.push_back(a);
            bs.iy.push_back(b);
            bs.iz.push_back(c);
        }
    }
    T.id = (int)P.trees.size();
    TreeDesc td{};
    td.target = target ? 1 : 0;
    td.rep = rep;
    td.H = H;
    for (int lv = 0; lv <= kMaxDepth; ++lv) T.off[lv] = -1;
    for (int lv = 2; lv <= H; ++lv) {
        int n = (int)T.B[lv].mkey.size();
        if (target) {
            T.off[lv] = P.n_le;
            P.n_le += n;
        } else {
            T.off[lv] = P.n_me;
            P.n_me += n;
        }
    }
    auto hlev = [&](int lv) { return 2.0 * R / (double)(1 << lv); };
    auto centre = [&](int lv, int i) { return -R + (i + 0.5) * hlev(lv); };   // canonical, relative to the root centre
    // leaves (leaf k is level-H box k); the points stay with the builder
    // (at most three point sets per charge on each side, and build_plan caps
    // the charges at 2^31 / 4: point indices fit in 32 bits)
    const int64_t g0 = target ? P.n_tpts : P.n_spts;
    std::vector<int>& lstart = target ? P.tl_start : P.sl_start;
    T.leaf0 = target ? (int)P.tl_le.size() : (int)P.sl_me.size();
    for (size_t k = 0; k < nl; ++k) {
        const int L = V.leaf_level(k, H);
        const uint64_t key = V.lkey[k];
        const int a = (int)morton_compact3(key >> 2), b = (int)morton_compact3(key >> 1), c = (int)morton_compact3(key);
        const int box = V.llv.empty() ? (int)k : T.B[L].find(a, b, c);
        if (k > 0) lstart.push_back((int)(g0 + V.lstart[k]));
        std::vector<int>& le = target ? P.tl_le : P.sl_me;
        le.push_back(L >= 2 ? T.off[L] + box : -1);
        (target ? P.tl_fmm : P.sl_fmm).push_back(rep);
        (target ? P.tl_tree : P.sl_tree).push_back(T.id);
        (target ? P.tl_h : P.sl_h).push_back(hlev(L));
        (target ? P.tl_lv : P.sl_lv).push_back(L);
        for (int v : {a, b, c}) (target ? P.tl_ctr : P.sl_ctr).push_back(centre(L, v));
        (target ? P.tl_cell : P.sl_cell).push_back(cellkey(a, b, c));
    }
    if (V.n > 0) lstart.push_back((int)(g0 + V.n));
    if (target) {
        P.t_sets.push_back(V.handle);
        P.t_set_slot.push_back(slot);
        P.n_tpts += V.n;
    } else {
        P.s_sets.push_back(V.handle);
        P.n_spts += V.n;
    }
    T.nleaf = (target ? (int)P.tl_le.size() : (int)P.sl_me.size()) - T.leaf0;
    td.leaf0 = T.leaf0;
    td.nleaf = T.nleaf;
    P.trees.push_back(td);
    // translation operators (b = child centre - parent centre) and their lists
    int lo = target ? 3 : 2, hi = target ? H : H - 1;
    for (int lv = lo; lv <= hi; ++lv) {
        double hc = hlev(target ? lv : lv + 1);
        int opo[8];
        for (int o = 0; o < 8; ++o) {
            OpDesc d{};
            d.type = target ? OP_L2L : OP_M2M;
            d.fmm = rep;
            d.level = lv;
            d.rkey = -1;
            d.bx = (((o >> 2) & 1) - 0.5) * hc;
            d.by = (((o >> 1) & 1) - 0.5) * hc;
            d.bz = ((o & 1) - 0.5) * hc;
            opo[o] = (int)P.ops.size();
            P.ops.push_back(d);
        }
        const int n = (int)T.B[lv].mkey.size();
        if (target) {
            // L2L: children of one octant share the operator; 64 per work item
            std::vector<int> byo[8];
            for (int k = 0; k < n; ++k) {
                int ix = T.B[lv].ix[k], iy = T.B[lv].iy[k], iz = T.B[lv].iz[k];
                byo[((ix & 1) << 2) | ((iy & 1) << 1) | (iz & 1)].push_back(k);
            }
            for (int o = 0; o < 8; ++o)
                for (size_t c0 = 0; c0 < byo[o].size(); c0 += 64) {
                    BWork wk;
                    wk.dst.fill(-1);
                    wk.op.assign(1, opo[o]);
                    wk.src.assign(64, -1);
                    for (size_t j = 0; j < 64 && c0 + j < byo[o].size(); ++j) {
                        int k = byo[o][c0 + j];
                        int ix = T.B[lv].ix[k], iy = T.B[lv].iy[k], iz = T.B[lv].iz[k];
                        wk.src[j] = T.off[lv - 1] + T.B[lv - 1].find(ix >> 1, iy >> 1, iz >> 1);
                        wk.dst[j] = T.off[lv] + k;
                    }
                    S.bl2l[lv].push_back(std::move(wk));
                }
        } else {
            // M2M: 64 parents per work item, one term per child octant (on
            // adaptive trees only the boxes with children: a leaf's expansion
            // comes from its P2M)
            std::vector<int> par;
            for (int k = 0; k < n; ++k) {
                const int px = T.B[lv].ix[k], py = T.B[lv].iy[k], pz = T.B[lv].iz[k];
                bool any = false;
                for (int o = 0; o < 8 && !any; ++o)
                    any = T.B[lv + 1].find(2 * px + ((o >> 2) & 1), 2 * py + ((o >> 1) & 1), 2 * pz + (o & 1)) >= 0;
                if (any) par.push_back(k);
            }
            const int npar = (int)par.size();
            for (int c0 = 0; c0 < npar; c0 += 64) {
                BWork wk;
                wk.dst.fill(-1);
                wk.op.assign(opo, opo + 8);
                wk.src.assign(8 * 64, -1);
                for (int j = 0; j < 64 && c0 + j < npar; ++j) {
                    int k = par[c0 + j];
                    int px = T.B[lv].ix[k], py = T.B[lv].iy[k], pz = T.B[lv].iz[k];
                    wk.dst[j] = T.off[lv] + k;
                    for (int o = 0; o < 8; ++o) {
                        const int ch = T.B[lv + 1].find(2 * px + ((o >> 2) & 1), 2 * py + ((o >> 1) & 1), 2 * pz + (o & 1));
                        if (ch >= 0) wk.src[64 * o + j] = T.off[lv + 1] + ch;
                    }
                }
                S.bm2m[lv].push_back(std::move(wk));
            }
        }
    }
}

// U-, W- and X-lists of one FMM on adaptive trees, by a dual traversal of its
// target and source trees from their roots (Sec. 3.5, closing remarks on
// adaptive trees; the V-list is the same rule as on uniform trees and comes
// from add_lists).  Pairs of adjacent boxes (levels below 2 count as
// adjacent: they carry no expansions) are refined: two leaves form a U-list
// pair; a target leaf and a source box with children: the children not
// adjacent to the leaf join its W-list (M2P), the others are refined; a
// source leaf and a target box with children: the children not adjacent to
// the leaf get the leaf in their X-list (P2L), the others are refined; two
// boxes with children: adjacent child pairs are refined (the others are
// V-list pairs).  Every (target, source) pair is then covered exactly once.
void adaptive_lists(Plan& P, Staging& S, int fid, const TreeB& ST, const TreeB& TT)
{
    const FmmDesc& F = P.fmm[fid];
    const int H = F.H;
    const double R = F.R;
    auto hlev = [&](int lv) { return 2.0 * R / (double)(1 << lv); };
    auto centre = [&](int lv, int i) { return -R + (i + 0.5) * hlev(lv); };
    const std::vector<BoxSet>& SB = ST.B;
    const std::vector<BoxSet>& TB = TT.B;
    const int hs = (int)SB.size() - 1, ht = (int)TB.size() - 1;
    // leaf index of each box (-1: the box has children)
    auto leaf_map = [&](const TreeB& T, const std::vector<int>& lvv, const std::vector<uint64_t>& cell) {
        std::vector<std::vector<int>> m(T.B.size());
        for (size_t l = 0; l < T.B.size(); ++l) m[l].assign(T.B[l].mkey.size(), -1);
        for (int i = T.leaf0; i < T.leaf0 + T.nleaf; ++i) {
            const uint64_t c = cell[i];
            const int a = (int)((c >> 42) & 0x1fffff), b = (int)((c >> 21) & 0x1fffff), z = (int)(c & 0x1fffff);
            m[lvv[i]][T.B[lvv[i]].find(a, b, z)] = i;
        }
        return m;
    };
    const std::vector<std::vector<int>> sleaf = leaf_map(ST, P.sl_lv, P.sl_cell);
    const std::vector<std::vector<int>> tleaf = leaf_map(TT, P.tl_lv, P.tl_cell);
    auto child = [](const std::vector<BoxSet>& B, int hb, int lv, int b, int o) {
        if (lv >= hb) return -1;
        return B[lv + 1].find(2 * B[lv].ix[b] + ((o >> 2) & 1), 2 * B[lv].iy[b] + ((o >> 1) & 1), 2 * B[lv].iz[b] + (o & 1));
    };
    auto adjacent = [&](int lt, int bt, int ls, int bs) {
        const int L = std::max(lt, ls);
        const int ct[3] = {TB[lt].ix[bt], TB[lt].iy[bt], TB[lt].iz[bt]};
        const int cs[3] = {SB[ls].ix[bs], SB[ls].iy[bs], SB[ls].iz[bs]};
        for (int d = 0; d < 3; ++d) {
            const int64_t tlo = (int64_t)ct[d] << (L - lt), thi = ((int64_t)(ct[d] + 1) << (L - lt)) - 1;
            const int64_t slo = (int64_t)cs[d] << (L - ls), shi = ((int64_t)(cs[d] + 1) << (L - ls)) - 1;
            if (tlo > shi + 1 || slo > thi + 1) return false;
        }
        return true;
    };
    std::vector<std::array<int, 2>> up;
    auto u_pair = [&](int tl, int sl) {
        const int64_t pairs = (int64_t)(P.tl_start[tl + 1] - P.tl_start[tl]) * (P.sl_start[sl + 1] - P.sl_start[sl]);
        P.n_p2p_pairs += pairs;
        if (F.kind == 1) P.n_react_p2p_pairs += pairs;
        up.push_back({tl, sl});
    };
    std::function<void(int, int, int, int)> refine = [&](int lt, int bt, int ls, int bs) {
        const int tl = tleaf[lt][bt], sl = sleaf[ls][bs];
        if (tl >= 0 && sl >= 0) {
            u_pair(tl, sl);
            return;
        }
        if (tl >= 0) {
            for (int o = 0; o < 8; ++o) {
                const int c = child(SB, hs, ls, bs, o);
                if (c < 0) continue;
                if (ls + 1 < 2 || adjacent(lt, bt, ls + 1, c)) refine(lt, bt, ls + 1, c);
                else {
                    S.w_pairs.push_back({tl, fid, ST.off[ls + 1] + c, ls + 1,
                                         {centre(ls + 1, SB[ls + 1].ix[c]), centre(ls + 1, SB[ls + 1].iy[c]),
                                          centre(ls + 1, SB[ls + 1].iz[c])}});
                    P.n_w_pairs++;
                }
            }
            return;
        }
        if (sl >= 0) {
            for (int o = 0; o < 8; ++o) {
                const int c = child(TB, ht, lt, bt, o);
                if (c < 0) continue;
                if (lt + 1 < 2 || adjacent(lt + 1, c, ls, bs)) refine(lt + 1, c, ls, bs);
                else {
                    S.x_pairs.push_back({TT.off[lt + 1] + c, lt + 1,
                                         {centre(lt + 1, TB[lt + 1].ix[c]), centre(lt + 1, TB[lt + 1].iy[c]),
                                          centre(lt + 1, TB[lt + 1].iz[c])},
                                         fid, sl});
                    P.n_x_pairs++;
                }
            }
            return;
        }
        for (int ot = 0; ot < 8; ++ot) {
            const int ct = child(TB, ht, lt, bt, ot);
            if (ct < 0) continue;
            for (int os = 0; os < 8; ++os) {
                const int cs = child(SB, hs, ls, bs, os);
                if (cs < 0) continue;
                if (lt + 1 < 2 || adjacent(lt + 1, ct, ls + 1, cs)) refine(lt + 1, ct, ls + 1, cs);
            }
        }
    };
    (void)H;
    if (!SB.empty() && !TB.empty() && !SB[0].mkey.empty() && !TB[0].mkey.empty()) refine(0, 0, 0, 0);
    // U-list entries grouped by target leaf; in free space (one point set,
    // source leaf k = target leaf k) a leaf's own leaf comes first, as the
    // near-field kernel expects
    auto rank = [&](const std::array<int, 2>& e) {
        const bool self = F.kind == 0 && e[1] - ST.leaf0 == e[0] - TT.leaf0;
        return (int64_t)e[0] * 2 + (self ? 0 : 1);
    };
    std::stable_sort(up.begin(), up.end(),
                     [&](const std::array<int, 2>& a, const std::array<int, 2>& b) { return rank(a) < rank(b); });
    for (const auto& e : up) {
        if (F.kind == 0) S.p2p_pairs.push_back({e[0], e[1]});
        else S.rp_pairs.push_back({e[0], fid, e[1]});
    }
}

// V-lists (M2L, with operator de-duplication and the tiled levels of a
// free-space FMM) and U-lists of one FMM between its source and target trees.
void add_lists(Plan& P, Staging& S, int fid, const TreeB& ST, const TreeB& TT)
{
    FmmDesc& F = P.fmm[fid];
    const int H = F.H;
    const double R = F.R;
    auto hlev = [&](int lv) { return 2.0 * R / (double)(1 << lv); };
    auto centre = [&](int lv, int i) { return -R + (i + 0.5) * hlev(lv); };
    const std::vector<BoxSet>& SB = ST.B;
    const std::vector<BoxSet>& TB = TT.B;
    // operator de-duplication: free-space operators per (level, offset), 343
    // offsets per level; reaction operators per (level, rho^2 / h^2, z cells),
    // where the z cells of a V-list pair lie within 3 of the interface plane
    // (targets above it, images below), so a small table per level serves
    // them, with a hash map as fallback
    std::vector<int> opmap((size_t)(kMaxDepth + 1) * 343, -1);
    constexpr int kRkD2 = 19, kRkZ = 4;
    std::vector<int> rktab((size_t)(kMaxDepth + 1) * kRkD2 * kRkZ * kRkZ, -1);
    std::unordered_map<uint64_t, int> rkmap;
    auto free_op = [&](int lv, int dx, int dy, int dz) {
        int& slot = opmap[(size_t)lv * 343 + ((dx + 3) * 7 + (dy + 3)) * 7 + (dz + 3)];
        if (slot >= 0) return slot;
        double h = hlev(lv);
        OpDesc d{};
        d.type = OP_M2L_FREE;
        d.fmm = fid;
        d.level = lv;
        d.rkey = -1;
        d.bx = -dx * h;   // b = c_t - c_s
        d.by = -dy * h;
        d.bz = -dz * h;
        int op = (int)P.ops.size();
        P.ops.push_back(d);
        slot = op;
        return op;
    };
    // tiled levels of a free-space FMM: dense grids, operator table, tiles
    // (in_tile[lv][box]: the target box belongs to a tile)
    std::vector<std::vector<char>> in_tile(kMaxDepth + 1);
    const int tiled_min = std::max(2, kTileMinLevel);
    const int tiled_max = (F.kind == 0) ? std::min(H, kTileMaxLevel) : 1;
    for (int lv = tiled_min; lv <= tiled_max; ++lv) {
        int nside = 1 << lv;
        TileFL t{};
        t.fmm = fid;
        t.level = lv;
        t.nside = nside;
        t.grid_off = (int)P.grid_me.size();
        t.optab_off = (int)P.optab.size();
        P.grid_me.resize(P.grid_me.size() + (size_t)nside * nside * nside, -1);
        P.grid_le.resize(P.grid_le.size() + (size_t)nside * nside * nside, -1);
        for (int k = 0; k < (int)SB[lv].mkey.size(); ++k)
            P.grid_me[t.grid_off + ((size_t)SB[lv].ix[k] * nside + SB[lv].iy[k]) * nside + SB[lv].iz[k]] = ST.off[lv] + k;
        for (int k = 0; k < (int)TB[lv].mkey.size(); ++k)
            P.grid_le[t.grid_off + ((size_t)TB[lv].ix[k] * nside + TB[lv].iy[k]) * nside + TB[lv].iz[k]] = TT.off[lv] + k;
        P.optab.resize(P.optab.size() + 343, -1);
        for (int dx = -3; dx <= 3; ++dx)
            for (int dy = -3; dy <= 3; ++dy)
                for (int dz = -3; dz <= 3; ++dz) {
                    if (std::abs(dx) <= 1 && std::abs(dy) <= 1 && std::abs(dz) <= 1) continue;
                    // reflection symmetry of the translation (real-form harmonics map to
                    // +- themselves under x, y or z -> -x, -y, -z): A_{sigma d} = D A_d D
                    const int refl = (dx < 0 ? 1 : 0) | (dy < 0 ? 2 : 0) | (dz < 0 ? 4 : 0);
                    P.optab[t.optab_off + ((dx + 3) * 7 + (dy + 3)) * 7 + (dz + 3)] =
                        free_op(lv, std::abs(dx), std::abs(dy), std::abs(dz)) | (refl << kReflShift);
                }
        int fl = (int)P.tfl.size();
        P.tfl.push_back(t);
        int np = nside / 2;
        std::vector<char>& mark = in_tile[lv];
        mark.assign(TB[lv].mkey.size(), 0);
        std::vector<int> boxes;
        for (int bx = 0; bx < np; bx += kTilePB)
            for (int by = 0; by < np; by += kTilePB)
                for (int bz = 0; bz < np; bz += kTilePB)
                    for (int o = 0; o < 8; ++o) {
                        boxes.clear();
                        for (int i = 0; i < kTilePB; ++i)
                            for (int j = 0; j < kTilePB; ++j)
                                for (int k = 0; k < kTilePB; ++k) {
                                    int tx = 2 * (bx + i) + ((o >> 2) & 1), ty = 2 * (by + j) + ((o >> 1) & 1),
                                        tz = 2 * (bz + k) + (o & 1);
                                    if (tx < nside && ty < nside && tz < nside) {
                                        const int le = P.grid_le[t.grid_off + ((size_t)tx * nside + ty) * nside + tz];
                                        if (le >= 0) boxes.push_back(le - TT.off[lv]);
                                    }
                                }
                        // a sparse tile's products are mostly padding: its target boxes'
                        // pairs go to the batched list instead
                        if ((int)boxes.size() < kTileMinBoxes) continue;
                        P.tiles.push_back({fl, o, bx, by, bz});
                        for (int b : boxes) mark[b] = 1;
                    }
    }
    for (int lv = 2; lv <= H; ++lv) {
        const bool tiled = lv >= tiled_min && lv <= tiled_max;
        int nside = 1 << lv;
        double h = hlev(lv);
        if (tiled) {
            // the tiles' operator tables cover these pairs: only their number
            // is needed, the non-empty source boxes among the children of the
            // parent's neighbours less those adjacent to the target, from
            // prefix sums of the source occupancy grid
            const int n1 = nside + 1;
            std::vector<int> ps((size_t)n1 * n1 * n1, 0);
            auto at = [&](int x, int y, int z) -> int& { return ps[((size_t)x * n1 + y) * n1 + z]; };
            for (size_t i = 0; i < SB[lv].mkey.size(); ++i) at(SB[lv].ix[i] + 1, SB[lv].iy[i] + 1, SB[lv].iz[i] + 1) = 1;
            for (int x = 1; x <= nside; ++x)
                for (int y = 1; y <= nside; ++y)
                    for (int z = 1; z <= nside; ++z) at(x, y, z) += at(x, y, z - 1);
            for (int x = 1; x <= nside; ++x)
                for (int y = 1; y <= nside; ++y)
                    for (int z = 1; z <= nside; ++z) at(x, y, z) += at(x, y - 1, z);
            for (int x = 1; x <= nside; ++x)
                for (int y = 1; y <= nside; ++y)
                    for (int z = 1; z <= nside; ++z) at(x, y, z) += at(x - 1, y, z);
            auto box = [&](int x0, int x1, int y0, int y1, int z0, int z1) {
                x0 = std::max(x0, 0); y0 = std::max(y0, 0); z0 = std::max(z0, 0);
                x1 = std::min(x1, nside - 1) + 1; y1 = std::min(y1, nside - 1) + 1; z1 = std::min(z1, nside - 1) + 1;
                if (x0 >= x1 || y0 >= y1 || z0 >= z1) return (int64_t)0;
                return (int64_t)at(x1, y1, z1) - at(x0, y1, z1) - at(x1, y0, z1) - at(x1, y1, z0) + at(x0, y0, z1) +
                       at(x0, y1, z0) + at(x1, y0, z0) - at(x0, y0, z0);
            };
            bool all = true;
            for (int k = 0; k < (int)TB[lv].mkey.size(); ++k) {
                if (!in_tile[lv][k]) {
                    all = false;
                    continue;
                }
                const int tx = TB[lv].ix[k], ty = TB[lv].iy[k], tz = TB[lv].iz[k];
                const int px = 2 * (tx >> 1), py = 2 * (ty >> 1), pz = 2 * (tz >> 1);
                const int64_t np = box(px - 2, px + 3, py - 2, py + 3, pz - 2, pz + 3) -
                                   box(tx - 1, tx + 1, ty - 1, ty + 1, tz - 1, tz + 1);
                P.n_m2l_tile_pairs += np;
                P.n_m2l_pairs += np;
            }
            if (all) continue;
            // the boxes of sparse tiles: listed below like an untiled level
        }
        // parents whose children can hold source boxes: those within the
        // cell range of the level's source boxes (a reaction FMM's images all
        // lie below the interface plane, so most targets have no V-list)
        int qlo[3] = {nside, nside, nside}, qhi[3] = {-1, -1, -1};
        for (size_t i = 0; i < SB[lv].mkey.size(); ++i) {
            const int c[3] = {SB[lv].ix[i] >> 1, SB[lv].iy[i] >> 1, SB[lv].iz[i] >> 1};
            for (int d = 0; d < 3; ++d) {
                qlo[d] = std::min(qlo[d], c[d]);
                qhi[d] = std::max(qhi[d], c[d]);
            }
        }
        for (int k = 0; k < (int)TB[lv].mkey.size(); ++k) {
            if (tiled && in_tile[lv][k]) continue;
            int tx = TB[lv].ix[k], ty = TB[lv].iy[k], tz = TB[lv].iz[k];
            int le = TT.off[lv] + k;
            const int qx0 = std::max((tx >> 1) - 1, qlo[0]), qx1 = std::min((tx >> 1) + 1, qhi[0]);
            const int qy0 = std::max((ty >> 1) - 1, qlo[1]), qy1 = std::min((ty >> 1) + 1, qhi[1]);
            const int qz0 = std::max((tz >> 1) - 1, qlo[2]), qz1 = std::min((tz >> 1) + 1, qhi[2]);
            for (int qx = qx0; qx <= qx1; ++qx)
                for (int qy = qy0; qy <= qy1; ++qy)
                    for (int qz = qz0; qz <= qz1; ++qz) {
                        for (int o = 0; o < 8; ++o) {
                            int sx = 2 * qx + ((o >> 2) & 1), sy = 2 * qy + ((o >> 1) & 1), sz = 2 * qz + (o & 1);
                            int dx = sx - tx, dy = sy - ty, dz = sz - tz;
                            if (std::abs(dx) <= 1 && std::abs(dy) <= 1 && std::abs(dz) <= 1) continue;
                            const int sbox = SB[lv].find(sx, sy, sz);
                            if (sbox < 0) continue;
                            int op, xc;
                            if (F.kind == 0) {
                                // one operator per offset with non-negative components, D A D for the others
                                op = free_op(lv, std::abs(dx), std::abs(dy), std::abs(dz));
                                xc = (dx < 0 ? 1 : 0) | (dy < 0 ? 2 : 0) | (dz < 0 ? 4 : 0);
                            } else {
                                // one operator per (level, rho, z_t, z_s) at phi = 0, rotated per pair
                                const int d2 = dx * dx + dy * dy;
                                const int zt_i = tz - nside / 2, zs_i = nside / 2 - 1 - sz;
                                int* rslot = nullptr;
                                if (d2 < kRkD2 && zt_i >= 0 && zt_i < kRkZ && zs_i >= 0 && zs_i < kRkZ)
                                    rslot = &rktab[(((size_t)lv * kRkD2 + d2) * kRkZ + zt_i) * kRkZ + zs_i];
                                const uint64_t rk = ((uint64_t)lv << 48) | ((uint64_t)d2 << 32) | ((uint64_t)tz << 16) | (uint64_t)sz;
                                int found = rslot ? *rslot : -1;
                                if (!rslot) {
                                    auto g = rkmap.find(rk);
                                    if (g != rkmap.end()) found = g->second;
                                }
                                if (found < 0) {
                                    RKey r{};
                                    r.fmm = fid;
                                    r.level = lv;
                                    r.rho = h * std::sqrt((double)d2);
                                    r.zt = centre(lv, tz);
                                    r.zs = centre(lv, sz);
                                    r.S = h;
                                    P.rkeys.push_back(r);
                                    OpDesc d{};
                                    d.type = OP_M2L_REACT;
                                    d.fmm = fid;
                                    d.level = lv;
                                    d.rkey = (int)P.rkeys.size() - 1;
                                    d.phi = 0.0;
                                    op = (int)P.ops.size();
                                    P.ops.push_back(d);
                                    if (rslot) *rslot = op;
                                    else rkmap[rk] = op;
                                } else op = found;
                                xc = kXfRotate + (dx + 3) * 7 + (dy + 3);
                            }
                            S.m2l_pairs.push_back({le, ST.off[lv] + sbox, op, xc});
                            P.n_m2l_pairs++;
                        }
                    }
        }
    }
    if (P.adaptive) {
        adaptive_lists(P, S, fid, ST, TT);
        return;
    }
    // U-lists at the leaf level (target leaf order equals the level-H box order);
    // the target's own box comes first
    int nside = 1 << H;
    static const int kUOrder[27][3] = {
        {0, 0, 0},   {-1, -1, -1}, {-1, -1, 0}, {-1, -1, 1}, {-1, 0, -1}, {-1, 0, 0}, {-1, 0, 1}, {-1, 1, -1}, {-1, 1, 0},
        {-1, 1, 1},  {0, -1, -1},  {0, -1, 0},  {0, -1, 1},  {0, 0, -1},  {0, 0, 1},  {0, 1, -1}, {0, 1, 0},   {0, 1, 1},
        {1, -1, -1}, {1, -1, 0},   {1, -1, 1},  {1, 0, -1},  {1, 0, 0},   {1, 0, 1},  {1, 1, -1}, {1, 1, 0},   {1, 1, 1}};
    int ulo[3] = {nside, nside, nside}, uhi[3] = {-1, -1, -1};
    for (size_t i = 0; i < SB[H].mkey.size(); ++i) {
        const int c[3] = {SB[H].ix[i], SB[H].iy[i], SB[H].iz[i]};
        for (int d = 0; d < 3; ++d) {
            ulo[d] = std::min(ulo[d], c[d]);
            uhi[d] = std::max(uhi[d], c[d]);
        }
    }
    for (int k = 0; k < TT.nleaf; ++k) {
        int tx = TB[H].ix[k], ty = TB[H].iy[k], tz = TB[H].iz[k];
        int tl = TT.leaf0 + k;
        int nt = P.tl_start[tl + 1] - P.tl_start[tl];
        // (no source leaf within one cell: empty U-list)
        if (tx + 1 < ulo[0] || tx - 1 > uhi[0] || ty + 1 < ulo[1] || ty - 1 > uhi[1] || tz + 1 < ulo[2] || tz - 1 > uhi[2])
            continue;
        for (const auto& du : kUOrder) {
                    int sx = tx + du[0], sy = ty + du[1], sz = tz + du[2];
                    if (sx < 0 || sy < 0 || sz < 0 || sx >= nside || sy >= nside || sz >= nside) continue;
                    const int sbox = SB[H].find(sx, sy, sz);
                    if (sbox < 0) continue;
                    int sl = ST.leaf0 + sbox;
                    int64_t pairs = (int64_t)nt * (P.sl_start[sl + 1] - P.sl_start[sl]);
                    P.n_p2p_pairs += pairs;
                    if (F.kind == 0) S.p2p_pairs.push_back({tl, sl});
                    else {
                        S.rp_pairs.push_back({tl, fid, sl});
                        P.n_react_p2p_pairs += pairs;
                    }
        }
    }
}

}  // namespace

std::string build_plan(Plan& P, const std::vector<Medium>& media, const std::vector<std::vector<double>>& xs,
                       const std::vector<std::vector<double>>& ys, const std::vector<std::vector<double>>& zs,
                       double iface_tol, PointBuilder& pb, int* status)
{
    const int cap = P.leaf_cap;
    *status = LPB_OK;
    P.nsys = (int)media.size();
    P.media = media;
    P.sys_charge_off.assign(P.nsys + 1, 0);
    for (int s = 0; s < P.nsys; ++s) P.sys_charge_off[s + 1] = P.sys_charge_off[s] + (int64_t)xs[s].size();
    P.ncharges = P.sys_charge_off[P.nsys];
    if (P.ncharges > (int64_t)0x7fffffff / 4) {
        *status = LPB_ERANGE;
        return "too many charges for 32-bit slot indices";
    }
    int maxL = 0;
    for (auto& m : media) maxL = std::max(maxL, m.L);
    // output slots: 0 free space, 1 reaction through the lower interface of
    // the target's layer (a = 1), 2 through the upper one (a = 2)
    P.nslots = maxL > 0 ? 3 : 1;
    P.fmm.clear();
    P.trees.clear();
    P.max_depth = 0;

    // ---- validation and layer classification ----
    std::vector<std::vector<int>> layer(P.nsys);
    for (int s = 0; s < P.nsys; ++s) {
        const Medium& m = media[s];
        layer[s].resize(xs[s].size());
        for (size_t i = 0; i < xs[s].size(); ++i) {
            double x = xs[s][i], y = ys[s][i], z = zs[s][i];
            if (!std::isfinite(x) || !std::isfinite(y) || !std::isfinite(z)) {
                *status = LPB_ENUMERIC;
                return "non-finite charge coordinate at index " + std::to_string(i);
            }
            for (int k = 0; k < m.L; ++k)
                if (std::fabs(z - m.d[k]) <= iface_tol) {
                    *status = LPB_ERANGE;
                    return "charge " + std::to_string(i) + " lies on interface " + std::to_string(k);
                }
            layer[s][i] = layer_of(m, z);
        }
    }

    // ---- accumulators of the plan ----
    P.n_spts = P.n_tpts = 0;
    P.s_sets.clear(); P.t_sets.clear(); P.t_set_slot.clear();
    P.sl_start.assign(1, 0); P.sl_me.clear(); P.sl_fmm.clear(); P.sl_tree.clear(); P.sl_h.clear();
    P.tl_start.assign(1, 0); P.tl_le.clear(); P.tl_fmm.clear(); P.tl_tree.clear(); P.tl_h.clear();
    P.sl_ctr.clear(); P.tl_ctr.clear(); P.sl_cell.clear(); P.tl_cell.clear();
    P.n_me = P.n_le = 0;
    P.ops.clear(); P.rkeys.clear();
    P.tfl.clear(); P.tiles.clear(); P.grid_me.clear(); P.grid_le.clear(); P.optab.clear();
    P.n_p2p_pairs = P.n_react_p2p_pairs = P.n_m2l_pairs = P.n_m2l_tile_pairs = 0;
    // V-list offsets of each child octant, grouped by reflection class (the
    // tiled kernel applies the sign flips once per run of equal class)
    P.oct_codes.clear();
    for (int o = 0; o < 8; ++o) {
        int ox = (o >> 2) & 1, oy = (o >> 1) & 1, oz = o & 1;
        std::vector<std::pair<int, int>> cl;
        for (int dx = -2 - ox; dx <= 3 - ox; ++dx)
            for (int dy = -2 - oy; dy <= 3 - oy; ++dy)
                for (int dz = -2 - oz; dz <= 3 - oz; ++dz) {
                    if (std::abs(dx) <= 1 && std::abs(dy) <= 1 && std::abs(dz) <= 1) continue;
                    int refl = (dx < 0 ? 1 : 0) | (dy < 0 ? 2 : 0) | (dz < 0 ? 4 : 0);
                    cl.push_back({refl, ((dx + 3) * 7 + (dy + 3)) * 7 + (dz + 3)});
                }
        std::stable_sort(cl.begin(), cl.end(), [](const std::pair<int, int>& a, const std::pair<int, int>& b) { return a.first < b.first; });
        for (auto& c : cl) P.oct_codes.push_back(c.second);
    }
    P.orb_tab.clear();
    for (int o = 0; o < 8; ++o) {
        const int oo[3] = {(o >> 2) & 1, (o >> 1) & 1, o & 1};
        std::vector<std::pair<int, std::vector<int>>> rows;   // (group rank, row)
        for (int a = 0; a <= 3; ++a)
            for (int b = 0; b <= 3; ++b)
                for (int c = 0; c <= 3; ++c) {
                    if (a <= 1 && b <= 1 && c <= 1) continue;
                    const int ad[3] = {a, b, c};
                    int both = 0, minus = 0;
                    for (int ax = 0; ax < 3; ++ax) {
                        // signs of this axis inside the octant's offset range [-2 - o, 3 - o]
                        const bool pos = ad[ax] <= 3 - oo[ax];
                        const bool neg = ad[ax] > 0 && -ad[ax] >= -2 - oo[ax];
                        if (pos && neg) both |= 1 << ax;
                        else if (neg) minus |= 1 << ax;
                    }
                    const int one = 7 & ~both;
                    auto deposit = [](int v, int mask) {
                        int r = 0;
                        for (int bit = 0; bit < 3; ++bit)
                            if ((mask >> bit) & 1) {
                                if (v & 1) r |= 1 << bit;
                                v >>= 1;
                            }
                        return r;
                    };
                    int nb = 0;
                    for (int ax = 0; ax < 3; ++ax) nb += (both >> ax) & 1;
                    int row[kOrbTab] = {};
                    row[0] = nb | (both << 4) | (minus << 7);
                    for (int j = 0; j < (1 << nb); ++j) {
                        const int sg = deposit(j, both) | minus;
                        int d[3];
                        for (int ax = 0; ax < 3; ++ax) d[ax] = ((sg >> ax) & 1) ? -ad[ax] : ad[ax];
                        row[1 + j] = ((d[0] + 3) * kOrbGrid + (d[1] + 3)) * kOrbGrid + (d[2] + 3);
                    }
                    for (int t = 0; t < (1 << (3 - nb)); ++t)
                        for (int j = 0; j < (1 << nb); ++j) {
                            const int g = deposit(j, both) | deposit(t, one);
                            int par = 0;
                            for (int bit = 0; bit < 3; ++bit) par ^= ((g & minus) >> bit) & 1;
                            row[9 + j + (t << nb)] = (int)(((unsigned)par << 31) | ((unsigned)g << 12));
                        }
                    row[17] = ((a + 3) * 7 + (b + 3)) * 7 + (c + 3);
                    int rank = 0;
                    while (kOrbGroupMask[rank] != both) ++rank;
                    rows.emplace_back(rank, std::vector<int>(row, row + kOrbTab));
                }
        std::stable_sort(rows.begin(), rows.end(),
                         [](const std::pair<int, std::vector<int>>& x, const std::pair<int, std::vector<int>>& y) { return x.first < y.first; });
        for (size_t q = 0; q < rows.size(); ++q) {
            if (rows.size() != (size_t)kOrbits || rows[q].first != (int)q / kOrbGroup) return "orbit groups: unexpected sizes";
            P.orb_tab.insert(P.orb_tab.end(), rows[q].second.begin(), rows[q].second.end());
        }
    }
    Staging S;

    for (int s = 0; s < P.nsys; ++s) {
        const Medium& m = media[s];
        const int L = m.L;
        const int64_t coff = P.sys_charge_off[s];
        std::vector<std::vector<int>> members(L + 1);
        for (size_t i = 0; i < xs[s].size(); ++i) members[layer[s][i]].push_back((int)i);
        auto base_desc = [&](int kind, int l, int lp, int a, int b) {
            FmmDesc F{};
            F.sys = s; F.kind = kind; F.l = l; F.lp = lp; F.a = a; F.b = b;
            F.lam_s = m.lam[lp];
            F.lam_t = m.lam[l];
            F.eps_t = m.eps[l];
            F.far_factor = (kind == 0) ? m.lam[l] / (2.0 * LPB_PI * LPB_PI * m.eps[l]) : 1.0;
            F.flip = (kind == 1 && a == 2) ? -1 : 1;
            F.layers_id = s;
            F.nsrc = (int)members[lp].size();
            F.ntgt = (int)members[l].size();
            return F;
        };

        // ---- free-space FMM of every layer: its own bounding cube and depth ----
        for (int l = 0; l <= L; ++l) {
            const auto& mem = members[l];
            if (mem.empty()) continue;
            FmmDesc F = base_desc(0, l, l, 0, 0);
            F.slot = 0;
            double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
            for (int i : mem) {
                double v[3] = {xs[s][i], ys[s][i], zs[s][i]};
                for (int d = 0; d < 3; ++d) { lo[d] = std::min(lo[d], v[d]); hi[d] = std::max(hi[d], v[d]); }
            }
            F.cx = 0.5 * (lo[0] + hi[0]);
            F.cy = 0.5 * (lo[1] + hi[1]);
            F.cz = 0.5 * (lo[2] + hi[2]);
            double r = 0.0;
            for (int d = 0; d < 3; ++d) r = std::max(r, 0.5 * (hi[d] - lo[d]));
            F.R = r > 0 ? r : 0.5;
            PtsInfo V;
            std::string msg;
            V.n = (int)mem.size();
            V.handle = pb.keys(s, coff, mem, SetFrame{0, 0, 0, F.cx, F.cy, F.cz}, F.R, V.counts, msg);
            if (V.handle < 0) {
                *status = pb.failure();
                return msg;
            }
            if (P.adaptive) {
                if (!pb.leaves_adaptive(V.handle, cap, false, V.lkey, V.llv, V.lstart, msg)) {
                    *status = pb.failure();
                    return msg;
                }
                F.H = V.max_level();
            } else {
                F.H = depth_rule(V, cap);
                if (!pb.leaves(V.handle, F.H, V.lkey, V.lstart, msg)) {
                    *status = pb.failure();
                    return msg;
                }
            }
            P.max_depth = std::max(P.max_depth, F.H);
            const int fid = (int)P.fmm.size();
            P.fmm.push_back(F);
            TreeB ST, TT;
            add_tree(P, S, V, F.H, F.R, false, fid, 0, ST);
            add_tree(P, S, V, F.H, F.R, true, fid, 0, TT);
            for (int lv = 0; lv <= kMaxDepth; ++lv) {
                P.fmm[fid].me_off[lv] = ST.off[lv];
                P.fmm[fid].le_off[lv] = TT.off[lv];
            }
            P.fmm[fid].src_tree = ST.id;
            P.fmm[fid].tgt_tree = TT.id;
            add_lists(P, S, fid, ST, TT);
        }
        if (L == 0) continue;

        // ---- reaction components: one grid for all of them ----
        // In the frame of a component (interface at z = 0, targets above it,
        // mirrored for a = 2) a target of layer l sits at +tau_a(z) and an
        // equivalent source of layer lp at -tau'_b(z') (eq. equivpolarcoord):
        // both depend only on their own layer and side, so each (layer, side)
        // point set has one source tree and one target tree, shared by all
        // components that use it, on a common root cube and depth.
        auto side_ok = [&](int l, int sd) { return sd == 1 ? l < L : l > 0; };
        auto tau = [&](int l, int sd, double z) { return sd == 1 ? z - m.d[l] : m.d[l - 1] - z; };
        double lo[2] = {INFINITY, INFINITY}, hi[2] = {-INFINITY, -INFINITY}, r = 0.0, tmin = INFINITY;
        for (size_t i = 0; i < xs[s].size(); ++i) {
            lo[0] = std::min(lo[0], xs[s][i]); hi[0] = std::max(hi[0], xs[s][i]);
            lo[1] = std::min(lo[1], ys[s][i]); hi[1] = std::max(hi[1], ys[s][i]);
            for (int sd = 1; sd <= 2; ++sd)
                if (side_ok(layer[s][i], sd)) {
                    double t = std::fabs(tau(layer[s][i], sd, zs[s][i]));
                    r = std::max(r, t);
                    tmin = std::min(tmin, t);
                }
        }
        if (xs[s].empty()) continue;
        const double gcx = 0.5 * (lo[0] + hi[0]), gcy = 0.5 * (lo[1] + hi[1]);
        r = std::max(r, 0.5 * (hi[0] - lo[0]));
        r = std::max(r, 0.5 * (hi[1] - lo[1]));
        const double R = r > 0 ? r : 0.5;
        // point sets: [l][sd][0 = images at -tau, 1 = targets at +tau]
        std::vector<std::array<std::array<PtsInfo, 2>, 3>> sets(L + 1);
        int H = 0;
        for (int l = 0; l <= L; ++l)
            for (int sd = 1; sd <= 2; ++sd) {
                if (!side_ok(l, sd) || members[l].empty()) continue;
                for (int tg = 0; tg < 2; ++tg) {
                    PtsInfo& V = sets[l][sd][tg];
                    std::string msg;
                    V.n = (int)members[l].size();
                    V.handle = pb.keys(s, coff, members[l], SetFrame{1, sd, tg, gcx, gcy, sd == 1 ? m.d[l] : m.d[l - 1]}, R,
                                       V.counts, msg);
                    if (V.handle < 0) {
                        *status = pb.failure();
                        return msg;
                    }
                    if (!P.adaptive) H = std::max(H, depth_rule(V, cap));
                }
            }
        // separation: leaves no wider than the smallest tau keep every target and
        // image one box away from the interface plane, so reaction U-lists are
        // empty (Remark 1); at most 3 levels above the occupancy depth.
        // Adaptive trees divide each set on its own: by occupancy and (mode 1)
        // by the same separation per box, up to 3 levels below occupancy.
        if (!P.adaptive) {
            int hs = 0;
            while (hs < kMaxDepth && 2.0 * R / (double)(1 << hs) > tmin) ++hs;
            hs = std::min(hs, std::min(H + 3, kMaxDepth));
            H = std::max(H, hs);
        }
        P.max_depth = std::max(P.max_depth, H);
        for (int l = 0; l <= L; ++l)
            for (int sd = 1; sd <= 2; ++sd)
                for (int tg = 0; tg < 2; ++tg) {
                    PtsInfo& V = sets[l][sd][tg];
                    std::string msg;
                    if (V.handle < 0) continue;
                    if (P.adaptive ? !pb.leaves_adaptive(V.handle, cap, P.adaptive == 1, V.lkey, V.llv, V.lstart, msg)
                                   : !pb.leaves(V.handle, H, V.lkey, V.lstart, msg)) {
                        *status = pb.failure();
                        return msg;
                    }
                    if (P.adaptive) H = std::max(H, V.max_level());
                }
        if (P.adaptive) P.max_depth = std::max(P.max_depth, H);
        // components in Algorithm 2 order
        std::vector<int> comp_fid;
        for (int a = 1; a <= 2; ++a)
            for (int b = 1; b <= 2; ++b)
                for (int l = (a == 1 ? 0 : 1); l < (a == 1 ? L : L + 1); ++l)
                    for (int lp = (b == 1 ? 0 : 1); lp < (b == 1 ? L : L + 1); ++lp) {
                        if (members[l].empty() || members[lp].empty()) continue;
                        FmmDesc F = base_desc(1, l, lp, a, b);
                        F.slot = a;
                        F.cx = gcx;
                        F.cy = gcy;
                        F.cz = (a == 1) ? m.d[l] : m.d[l - 1];
                        F.R = R;
                        F.H = H;
                        comp_fid.push_back((int)P.fmm.size());
                        P.fmm.push_back(F);
                    }
        // shared trees; the first component using a tree lends it lambda and root
        std::vector<std::array<TreeB, 3>> src_t(L + 1), tgt_t(L + 1);
        for (int fid : comp_fid) {
            FmmDesc& F = P.fmm[fid];
            if (src_t[F.lp][F.b].id < 0) add_tree(P, S, sets[F.lp][F.b][0], H, R, false, fid, 0, src_t[F.lp][F.b]);
            if (tgt_t[F.l][F.a].id < 0) add_tree(P, S, sets[F.l][F.a][1], H, R, true, fid, F.a, tgt_t[F.l][F.a]);
        }
        for (int fid : comp_fid) {
            FmmDesc& F = P.fmm[fid];
            const TreeB& ST = src_t[F.lp][F.b];
            const TreeB& TT = tgt_t[F.l][F.a];
            for (int lv = 0; lv <= kMaxDepth; ++lv) {
                F.me_off[lv] = ST.off[lv];
                F.le_off[lv] = TT.off[lv];
            }
            F.src_tree = ST.id;
            F.tgt_tree = TT.id;
            add_lists(P, S, fid, ST, TT);
        }
    }
    // ---- finalise flattened arrays ----
    // CSR by LE box, each box's pairs in the order they were listed (a stable
    // counting sort of the pair list by box)
    P.m2l_ptr.assign((size_t)P.n_le + 1, 0);
    for (const auto& e : S.m2l_pairs) P.m2l_ptr[e.le + 1]++;
    for (int i = 0; i < P.n_le; ++i) P.m2l_ptr[i + 1] += P.m2l_ptr[i];
    P.m2l_src.resize(S.m2l_pairs.size());
    P.m2l_op.resize(S.m2l_pairs.size());
    P.m2l_xc.resize(S.m2l_pairs.size());
    {
        std::vector<int> fill(P.m2l_ptr.begin(), P.m2l_ptr.end() - 1);
        for (const auto& e : S.m2l_pairs) {
            const int k = fill[e.le]++;
            P.m2l_src[k] = e.src;
            P.m2l_op[k] = e.op;
            P.m2l_xc[k] = e.xc;
        }
    }
    S.m2l_pairs = std::vector<Staging::M2LPair>();
    // batched work items: M2M and L2L per level, then the V-list pairs outside
    // the tiled levels grouped by operator
    P.bw_term_ptr.assign(1, 0); P.bw_op.clear(); P.bw_src.clear(); P.bw_dst.clear(); P.bw_xc.clear();
    auto push_work = [&](const BWork& wk) {
        P.bw_op.insert(P.bw_op.end(), wk.op.begin(), wk.op.end());
        P.bw_src.insert(P.bw_src.end(), wk.src.begin(), wk.src.end());
        P.bw_dst.insert(P.bw_dst.end(), wk.dst.begin(), wk.dst.end());
        P.bw_xc.insert(P.bw_xc.end(), wk.xc.begin(), wk.xc.end());
        P.bw_term_ptr.push_back((int)P.bw_op.size());
    };
    P.bm2m_lv.assign(kMaxDepth + 2, 0);
    P.bl2l_lv.assign(kMaxDepth + 2, 0);
    for (int lv = 0; lv <= kMaxDepth; ++lv) {
        P.bm2m_lv[lv] = (int)P.bw_term_ptr.size() - 1;
        for (auto& wk : S.bm2m[lv]) push_work(wk);
    }
    P.bm2m_lv[kMaxDepth + 1] = (int)P.bw_term_ptr.size() - 1;
    for (int lv = 0; lv <= kMaxDepth; ++lv) {
        P.bl2l_lv[lv] = (int)P.bw_term_ptr.size() - 1;
        for (auto& wk : S.bl2l[lv]) push_work(wk);
    }
    P.bl2l_lv[kMaxDepth + 1] = (int)P.bw_term_ptr.size() - 1;
    P.bm2l_w0 = (int)P.bw_term_ptr.size() - 1;
    {
        // (op, pair position) in increasing order: a counting sort by operator
        // (stable, so positions stay increasing within an operator)
        std::vector<std::pair<int, int>> byop(P.m2l_op.size());
        {
            std::vector<int> start(P.ops.size() + 1, 0);
            for (int op : P.m2l_op) start[op + 1]++;
            for (size_t i = 0; i < P.ops.size(); ++i) start[i + 1] += start[i];
            for (size_t k = 0; k < P.m2l_op.size(); ++k) byop[start[P.m2l_op[k]]++] = {P.m2l_op[k], (int)k};
        }
        // one term of up to 64 pairs per item, written straight into the arrays
        {
            size_t items = 0;
            for (size_t i = 0; i < byop.size();) {
                size_t e = i;
                while (e < byop.size() && e - i < 64 && byop[e].first == byop[i].first) ++e;
                ++items;
                i = e;
            }
            P.bw_op.reserve(P.bw_op.size() + items);
            P.bw_term_ptr.reserve(P.bw_term_ptr.size() + items);
            P.bw_src.reserve(P.bw_src.size() + 64 * items);
            P.bw_dst.reserve(P.bw_dst.size() + 64 * items);
            P.bw_xc.reserve(P.bw_xc.size() + 64 * items);
        }
        for (size_t i = 0; i < byop.size();) {
            size_t e = i;
            while (e < byop.size() && e - i < 64 && byop[e].first == byop[i].first) ++e;
            P.bw_op.push_back(byop[i].first);
            const size_t s0 = P.bw_src.size(), d0 = P.bw_dst.size();
            P.bw_src.resize(s0 + 64, -1);
            P.bw_dst.resize(d0 + 64, -1);
            P.bw_xc.resize(d0 + 64, -1);
            for (size_t j = i; j < e; ++j) {
                P.bw_src[s0 + j - i] = P.m2l_src[byop[j].second];
                P.bw_dst[d0 + j - i] = byop[j].second;
                P.bw_xc[d0 + j - i] = P.m2l_xc[byop[j].second];
            }
            P.bw_term_ptr.push_back((int)P.bw_op.size());
            i = e;
        }
    }
    P.bm2l_w1 = (int)P.bw_term_ptr.size() - 1;
    // canonical operators of the tiled levels (the orbit kernel's operands)
    P.orb_ops.clear();
    P.orb_index.assign(P.ops.size(), -1);
    for (const TileFL& t : P.tfl)
        for (int q = 0; q < kOrbits; ++q) {
            const int op = P.optab[t.optab_off + P.orb_tab[q * kOrbTab + 17]] & ((1 << kReflShift) - 1);
            if (P.orb_index[op] < 0) {
                P.orb_index[op] = (int)P.orb_ops.size();
                P.orb_ops.push_back(op);
            }
        }
    // every operator is stored in the MFMA operand layout
    P.swz_ops.resize(P.ops.size());
    P.swz_index.resize(P.ops.size());
    for (size_t i = 0; i < P.ops.size(); ++i) P.swz_ops[i] = P.swz_index[i] = (int)i;
    // W-lists: CSR by target leaf; X-lists: by target LE box (boxes in order of
    // first appearance), entries in the order found; reaction entries get
    // their point operators (one per point of the leaf on the point side)
    {
        const size_t nt = P.tl_le.size();
        const int K = P.K;
        P.w_ptr.assign(nt + 1, 0);
        for (const auto& e : S.w_pairs) P.w_ptr[e.tl + 1]++;
        for (size_t t = 0; t < nt; ++t) P.w_ptr[t + 1] += P.w_ptr[t];
        const size_t nw = S.w_pairs.size();
        P.w_fmm.resize(nw);
        P.w_me.resize(nw);
        P.w_lv.resize(nw);
        P.w_ctr.resize(3 * nw);
        P.w_vec.assign(nw, -1);
        std::vector<int> fill(P.w_ptr.begin(), P.w_ptr.end() - 1);
        int64_t vec = 0;
        for (const auto& e : S.w_pairs) {
            const int k = fill[e.tl]++;
            P.w_fmm[k] = e.fmm;
            P.w_me[k] = e.me;
            P.w_lv[k] = e.lv;
            for (int d = 0; d < 3; ++d) P.w_ctr[3 * k + d] = e.c[d];
        }
        for (size_t t = 0; t < nt; ++t)
            for (int k = P.w_ptr[t]; k < P.w_ptr[t + 1]; ++k) {
                const int n = P.tl_start[t + 1] - P.tl_start[t];
                P.n_w_points += n;
                if (P.fmm[P.w_fmm[k]].kind != 1) continue;
                P.w_vec[k] = vec;
                const double h = 2.0 * P.fmm[P.w_fmm[k]].R / (double)(1 << P.w_lv[k]);
                for (int j = 0; j < n; ++j) {
                    P.pt_ops.push_back({0, P.w_fmm[k], P.tl_start[t] + j, (int)t, P.w_ctr[3 * k], P.w_ctr[3 * k + 1],
                                        P.w_ctr[3 * k + 2], h, vec});
                    vec += K;
                }
            }
        std::unordered_map<int, int> box_of;
        std::vector<int> cnt;
        for (const auto& e : S.x_pairs) {
            auto it = box_of.find(e.le);
            if (it == box_of.end()) {
                box_of[e.le] = (int)P.x_box_le.size();
                P.x_box_le.push_back(e.le);
                P.x_box_lv.push_back(e.lv);
                for (int d = 0; d < 3; ++d) P.x_box_ctr.push_back(e.c[d]);
                cnt.push_back(0);
            }
            cnt[box_of[e.le]]++;
        }
        const size_t nb = P.x_box_le.size();
        P.x_box_ptr.assign(nb + 1, 0);
        for (size_t b = 0; b < nb; ++b) P.x_box_ptr[b + 1] = P.x_box_ptr[b] + cnt[b];
        const size_t nx = S.x_pairs.size();
        P.x_fmm.resize(nx);
        P.x_sl.resize(nx);
        P.x_vec.assign(nx, -1);
        std::vector<int> xf(P.x_box_ptr.begin(), P.x_box_ptr.end() - 1);
        for (const auto& e : S.x_pairs) {
            const int k = xf[box_of[e.le]]++;
            P.x_fmm[k] = e.fmm;
            P.x_sl[k] = e.sl;
        }
        for (size_t b = 0; b < nb; ++b)
            for (int k = P.x_box_ptr[b]; k < P.x_box_ptr[b + 1]; ++k) {
                const int sl = P.x_sl[k];
                const int n = P.sl_start[sl + 1] - P.sl_start[sl];
                P.n_x_points += n;
                if (P.fmm[P.x_fmm[k]].kind != 1) continue;
                P.x_vec[k] = vec;
                const double h = 2.0 * P.fmm[P.x_fmm[k]].R / (double)(1 << P.x_box_lv[b]);
                for (int j = 0; j < n; ++j) {
                    P.pt_ops.push_back({1, P.x_fmm[k], P.sl_start[sl] + j, sl, P.x_box_ctr[3 * b],
                                        P.x_box_ctr[3 * b + 1], P.x_box_ctr[3 * b + 2], h, vec});
                    vec += K;
                }
            }
    }
    // U-lists: CSR by target leaf, each leaf's entries in the order found (a
    // stable counting sort)
    {
        const size_t nt = P.tl_le.size();
        P.p2p_ptr.assign(nt + 1, 0);
        for (const auto& e : S.p2p_pairs) P.p2p_ptr[e[0] + 1]++;
        for (size_t t = 0; t < nt; ++t) P.p2p_ptr[t + 1] += P.p2p_ptr[t];
        P.p2p_src.resize(S.p2p_pairs.size());
        std::vector<int> fill(P.p2p_ptr.begin(), P.p2p_ptr.end() - 1);
        for (const auto& e : S.p2p_pairs) P.p2p_src[fill[e[0]]++] = e[1];
        P.rp_ptr.assign(nt + 1, 0);
        for (const auto& e : S.rp_pairs) P.rp_ptr[e[0] + 1]++;
        for (size_t t = 0; t < nt; ++t) P.rp_ptr[t + 1] += P.rp_ptr[t];
        P.rp_fmm.resize(S.rp_pairs.size());
        P.rp_src.resize(S.rp_pairs.size());
        fill.assign(P.rp_ptr.begin(), P.rp_ptr.end() - 1);
        for (const auto& e : S.rp_pairs) {
            const int k = fill[e[0]]++;
            P.rp_fmm[k] = e[1];
            P.rp_src[k] = e[2];
        }
    }
    return "";
}

uint64_t leaf_key(uint64_t lcell, int H, int flip)
{
    uint32_t a = (uint32_t)(lcell >> 42) & 0x1fffffu, b = (uint32_t)(lcell >> 21) & 0x1fffffu, c = (uint32_t)lcell & 0x1fffffu;
    if (flip < 0) c = (uint32_t)((1 << H) - 1) - c;
    return morton(a, b, c, H);
}

// ---------------------------------------------------------------------------
// Gaunt integrals from Wigner 3j symbols (Racah's formula, long double):
//   int Y^s_{l1 m1} Y^s_{l2 m2} Y^s_{l3 m3} = sqrt((2l1+1)(2l2+1)(2l3+1)/(4 pi))
//                                         (l1 l2 l3; 0 0 0) (l1 l2 l3; m1 m2 m3)
// for Condon-Shortley harmonics Y^s; the library's harmonics are
// Y_n^m = (-1)^m Y^s_{nm}, hence the extra (-1)^{m1+m2+m3} (= 1 when the
// integral is non-zero, since m1+m2+m3 = 0).
// ---------------------------------------------------------------------------
static long double lfact(int n)
{
    static long double tab[200];
    static bool init = false;
    if (!init) {
        tab[0] = 1.0L;
        for (int k = 1; k < 200; ++k) tab[k] = tab[k - 1] * (long double)k;
        init = true;
    }
    return tab[n];
}

static long double wigner3j(int j1, int j2, int j3, int m1, int m2, int m3)
{
    if (m1 + m2 + m3 != 0) return 0.0L;
    if (j3 < std::abs(j1 - j2) || j3 > j1 + j2) return 0.0L;
    if (std::abs(m1) > j1 || std::abs(m2) > j2 || std::abs(m3) > j3) return 0.0L;
    long double tri = lfact(j1 + j2 - j3) * lfact(j1 - j2 + j3) * lfact(-j1 + j2 + j3) / lfact(j1 + j2 + j3 + 1);
    long double pre = std::sqrt(tri * lfact(j1 + m1) * lfact(j1 - m1) * lfact(j2 + m2) * lfact(j2 - m2) * lfact(j3 + m3) *
                                lfact(j3 - m3));
    int kmin = std::max(0, std::max(j2 - j3 - m1, j1 - j3 + m2));
    int kmax = std::min(j1 + j2 - j3, std::min(j1 - m1, j2 + m2));
    long double sum = 0.0L;
    for (int k = kmin; k <= kmax; ++k) {
        long double den = lfact(k) * lfact(j3 - j2 + k + m1) * lfact(j3 - j1 + k - m2) * lfact(j1 + j2 - j3 - k) *
                          lfact(j1 - k - m1) * lfact(j2 - k + m2);
        sum += ((k & 1) ? -1.0L : 1.0L) / den;
    }
    int ph = j1 - j2 - m3;
    return ((ph & 1) ? -1.0L : 1.0L) * pre * sum;
}

double host_gaunt(int n1, int m1, int n2, int m2, int n3, int m3)
{
    if (m1 + m2 + m3 != 0) return 0.0;
    long double w0 = wigner3j(n1, n2, n3, 0, 0, 0);
    if (w0 == 0.0L) return 0.0;
    long double w = wigner3j(n1, n2, n3, m1, m2, m3);
    long double pre = std::sqrt((2.0L * n1 + 1) * (2.0L * n2 + 1) * (2.0L * n3 + 1) / (4.0L * 3.14159265358979323846264338327950288L));
    return (double)(pre * w0 * w);
}

}  // namespace lpb
