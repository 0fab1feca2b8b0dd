// lpb_plan.cpp -- host construction of the FMM plan: layers of the charges,
// equivalent polarization coordinates, one uniform octree per FMM, the
// interaction lists and the operator descriptors.
//
// Tree rule (identical in meaning to the oracle's, written independently):
//   root cube: free space -> centre of the bounding box of the layer's
//     charges, half side = half the largest extent; reaction -> centred in z
//     on the interface between targets and images (Sec. 3.5: the largest box
//     is divided in half by that interface), centred in x,y on the bounding
//     box of targets and sources, half side = max of |z - interface| and the
//     half x,y extents.
//   fine cell per axis: floor(((x - c) + R) / (2R) * 65536) clamped to
//     [0, 65535]; the level-l cell is the fine cell >> (16 - l).
//   depth H: smallest l (<= 12) with N_src <= cap * (non-empty source boxes at
//     l) and N_tgt <= cap * (non-empty target boxes at l).
//   V-list (levels >= 2): source boxes that are children of the neighbours
//     of the target's parent and not adjacent to the target; U-list at level
//     H: the target's neighbours and itself.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <unordered_map>

#include "lpb_internal.h"

namespace lpb {

namespace {

uint32_t fine_cell(double x, double c, double R)
{
    double t = ((x - c) + R) / (2.0 * R);
    double f = std::floor(t * 65536.0);
    if (!(f >= 0.0)) f = 0.0;
    if (f > 65535.0) f = 65535.0;
    return (uint32_t)f;
}

// Morton key of a level-l cell: bits interleaved x, y, z from the top level down.
uint64_t morton(uint32_t ix, uint32_t iy, uint32_t iz, int l)
{
    uint64_t k = 0;
    for (int bit = l - 1; bit >= 0; --bit)
        k = (k << 3) | ((uint64_t)((ix >> bit) & 1u) << 2) | ((uint64_t)((iy >> bit) & 1u) << 1) |
            (uint64_t)((iz >> bit) & 1u);
    return k;
}

// spread the low 16 bits of v to every third bit
inline uint64_t spread3(uint32_t v)
{
    uint64_t x = v & 0xffffu;
    x = (x | (x << 16)) & 0x0000ff0000ffull;
    x = (x | (x << 8)) & 0x00f00f00f00full;
    x = (x | (x << 4)) & 0x0c30c30c30c3ull;
    x = (x | (x << 2)) & 0x249249249249ull;
    return x;
}

// Morton key of a fine cell (16 levels): same bit order as morton(.., 16)
inline uint64_t morton_fine(uint32_t ix, uint32_t iy, uint32_t iz) { return (spread3(ix) << 2) | (spread3(iy) << 1) | spread3(iz); }

inline uint64_t cellkey(int ix, int iy, int iz)
{
    return ((uint64_t)(uint32_t)ix << 42) | ((uint64_t)(uint32_t)iy << 21) | (uint64_t)(uint32_t)iz;
}

struct Pt {
    uint64_t fkey;   // Morton key of the fine cell (canonical frame)
    uint32_t c[3];   // fine cells (canonical frame)
    double x, y, z;  // original frame (z = image z for reaction sources)
    int cidx;        // global charge index
    int local;       // index within the system
};

bool comp_valid(int L, int l, int lp, int a, int b)
{
    if (a == 1 && l >= L) return false;
    if (a == 2 && l <= 0) return false;
    if (b == 1 && lp >= L) return false;
    if (b == 2 && lp <= 0) return false;
    return true;
}

struct BoxSet {
    // level-l boxes of one point set: canonical cell coords sorted by Morton key
    std::vector<uint64_t> mkey;
    std::vector<int> ix, iy, iz;
    std::unordered_map<uint64_t, int> idx;   // cellkey -> position
};

}  // namespace

std::string build_plan(Plan& P, const std::vector<Medium>& media, const std::vector<std::vector<double>>& xs,
                       const std::vector<std::vector<double>>& ys, const std::vector<std::vector<double>>& zs,
                       double iface_tol, int* status)
{
    const int p = P.p;
    const int cap = P.leaf_cap;
    *status = LPB_OK;
    P.nsys = (int)media.size();
    P.media = media;
    P.sys_charge_off.assign(P.nsys + 1, 0);
    for (int s = 0; s < P.nsys; ++s) P.sys_charge_off[s + 1] = P.sys_charge_off[s] + (int64_t)xs[s].size();
    P.ncharges = P.sys_charge_off[P.nsys];
    if (P.ncharges > (int64_t)0x7fffffff / 16) {
        *status = LPB_ERANGE;
        return "too many charges for 32-bit slot indices";
    }
    int maxL = 0;
    for (auto& m : media) maxL = std::max(maxL, m.L);
    P.nslots = 1 + 4 * maxL;
    P.fmm.clear();
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
    P.s_cidx.clear(); P.t_cidx.clear(); P.s_u.clear(); P.t_u.clear(); P.t_out.clear();
    P.sl_start.assign(1, 0); P.sl_me.clear(); P.sl_fmm.clear(); P.sl_level.clear(); P.sl_h.clear();
    P.tl_start.assign(1, 0); P.tl_le.clear(); P.tl_fmm.clear(); P.tl_h.clear();
    P.sl_ctr.clear(); P.tl_ctr.clear(); P.s_okey.clear(); P.t_okey.clear();
    P.me_fmm.clear(); P.me_level.clear(); P.le_fmm.clear(); P.le_level.clear();
    P.n_me = P.n_le = 0;
    P.ops.clear(); P.rkeys.clear();
    P.tfl.clear(); P.tiles.clear(); P.grid_me.clear(); P.grid_le.clear(); P.optab.clear();
    P.n_p2p_pairs = P.n_react_p2p_pairs = P.n_m2l_pairs = P.n_m2l_tile_pairs = 0;
    P.oct_codes.clear();
    for (int o = 0; o < 8; ++o) {
        int ox = (o >> 2) & 1, oy = (o >> 1) & 1, oz = o & 1;
        for (int dx = -2 - ox; dx <= 3 - ox; ++dx)
            for (int dy = -2 - oy; dy <= 3 - oy; ++dy)
                for (int dz = -2 - oz; dz <= 3 - oz; ++dz) {
                    if (std::abs(dx) <= 1 && std::abs(dy) <= 1 && std::abs(dz) <= 1) continue;
                    P.oct_codes.push_back(((dx + 3) * 7 + (dy + 3)) * 7 + (dz + 3));
                }
    }
    // per-level staging (levels are contiguous across FMMs in the final arrays)
    struct M2MRec { int parent, child, op; };
    struct L2LRec { int child, parent, op; };
    std::vector<std::vector<M2MRec>> m2m_by_level(kMaxDepth + 1);
    std::vector<std::vector<L2LRec>> l2l_by_level(kMaxDepth + 1);
    std::vector<std::vector<std::pair<int, int>>> m2l_by_le;   // per LE box: (src ME, op)
    std::vector<std::vector<int>> p2p_by_tl;                    // per target leaf: source leaves
    std::vector<double> s_ux, s_uy, s_uz, t_ux, t_uy, t_uz;

    for (int s = 0; s < P.nsys; ++s) {
        const Medium& m = media[s];
        const int L = m.L;
        const int64_t coff = P.sys_charge_off[s];
        // components in Algorithm 2 order
        struct C { int kind, l, lp, a, b; };
        std::vector<C> comps;
        for (int l = 0; l <= L; ++l) comps.push_back({0, l, l, 0, 0});
        for (int a = 1; a <= 2; ++a)
            for (int b = 1; b <= 2; ++b)
                for (int l = (a == 1 ? 0 : 1); l < (a == 1 ? L : L + 1); ++l)
                    for (int lp = (b == 1 ? 0 : 1); lp < (b == 1 ? L : L + 1); ++lp) comps.push_back({1, l, lp, a, b});
        std::vector<int> slot_ctr(L + 1, 1);
        std::vector<std::vector<int>> members(L + 1);
        for (size_t i = 0; i < xs[s].size(); ++i) members[layer[s][i]].push_back((int)i);

        for (const C& cp : comps) {
            int slot = (cp.kind == 0) ? 0 : slot_ctr[cp.l]++;
            const auto& tgt = members[cp.l];
            const auto& src = members[cp.lp];
            if (tgt.empty() || src.empty()) continue;
            FmmDesc F{};
            F.sys = s;
            F.kind = cp.kind;
            F.l = cp.l;
            F.lp = cp.lp;
            F.a = cp.a;
            F.b = cp.b;
            F.slot = slot;
            F.lam_s = m.lam[cp.lp];
            F.lam_t = m.lam[cp.l];
            F.eps_t = m.eps[cp.l];
            F.far_factor = (cp.kind == 0) ? m.lam[cp.l] / (2.0 * LPB_PI * LPB_PI * m.eps[cp.l]) : 1.0;
            F.flip = (cp.kind == 1 && cp.a == 2) ? -1 : 1;
            F.layers_id = s;
            // points; reaction sources are images (eq. equivpolarcoord, with the source's own z)
            std::vector<Pt> T(tgt.size()), S(src.size());
            for (size_t k = 0; k < tgt.size(); ++k) {
                int i = tgt[k];
                T[k].x = xs[s][i]; T[k].y = ys[s][i]; T[k].z = zs[s][i];
                T[k].cidx = (int)(coff + i);
                T[k].local = i;
            }
            double zi = 0.0;
            if (cp.kind == 1) zi = (cp.a == 1) ? m.d[cp.l] : m.d[cp.l - 1];
            for (size_t k = 0; k < src.size(); ++k) {
                int i = src[k];
                S[k].x = xs[s][i]; S[k].y = ys[s][i];
                double z = zs[s][i];
                if (cp.kind == 1) {
                    double ts = (cp.b == 1) ? z - m.d[cp.lp] : m.d[cp.lp - 1] - z;
                    z = (cp.a == 1) ? m.d[cp.l] - ts : m.d[cp.l - 1] + ts;
                }
                S[k].z = z;
                S[k].cidx = (int)(coff + i);
                S[k].local = i;
            }
            // root cube
            if (cp.kind == 0) {
                double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
                for (auto& q : T) {
                    double v[3] = {q.x, q.y, q.z};
                    for (int d = 0; d < 3; ++d) { lo[d] = std::min(lo[d], v[d]); hi[d] = std::max(hi[d], v[d]); }
                }
                F.cx = 0.5 * (lo[0] + hi[0]);
                F.cy = 0.5 * (lo[1] + hi[1]);
                F.cz = 0.5 * (lo[2] + hi[2]);
                double r = 0.0;
                for (int d = 0; d < 3; ++d) r = std::max(r, 0.5 * (hi[d] - lo[d]));
                F.R = r > 0 ? r : 0.5;
            } else {
                double lo[2] = {INFINITY, INFINITY}, hi[2] = {-INFINITY, -INFINITY};
                double r = 0.0;
                for (auto* V : {&T, &S})
                    for (auto& q : *V) {
                        lo[0] = std::min(lo[0], q.x); hi[0] = std::max(hi[0], q.x);
                        lo[1] = std::min(lo[1], q.y); hi[1] = std::max(hi[1], q.y);
                        r = std::max(r, std::fabs(q.z - zi));
                    }
                F.cx = 0.5 * (lo[0] + hi[0]);
                F.cy = 0.5 * (lo[1] + hi[1]);
                F.cz = zi;
                r = std::max(r, 0.5 * (hi[0] - lo[0]));
                r = std::max(r, 0.5 * (hi[1] - lo[1]));
                F.R = r > 0 ? r : 0.5;
            }
            for (auto* V : {&T, &S})
                for (auto& q : *V) {
                    q.c[0] = fine_cell(q.x, F.cx, F.R);
                    q.c[1] = fine_cell(q.y, F.cy, F.R);
                    q.c[2] = fine_cell(q.z, F.cz, F.R);
                    if (F.flip < 0) q.c[2] = 65535u - q.c[2];   // canonical frame: mirror z
                }
            // fine Morton keys; one sort per point set, then every level is a prefix
            for (auto* V : {&T, &S})
                for (auto& q : *V) q.fkey = morton_fine(q.c[0], q.c[1], q.c[2]);
            auto byfine = [](const Pt& A, const Pt& B) { return A.fkey != B.fkey ? A.fkey < B.fkey : A.cidx < B.cidx; };
            std::sort(T.begin(), T.end(), byfine);
            std::sort(S.begin(), S.end(), byfine);
            auto count_level = [](const std::vector<Pt>& V, int lv) {
                int sh = 3 * (kCellBits - lv);
                int64_t n = V.empty() ? 0 : 1;
                for (size_t i = 1; i < V.size(); ++i)
                    if ((V[i].fkey >> sh) != (V[i - 1].fkey >> sh)) ++n;
                return n;
            };
            // depth
            int H = kMaxDepth;
            for (int lv = 0; lv <= kMaxDepth; ++lv) {
                if ((int64_t)S.size() <= (int64_t)cap * count_level(S, lv) &&
                    (int64_t)T.size() <= (int64_t)cap * count_level(T, lv)) {
                    H = lv;
                    break;
                }
            }
            F.H = H;
            P.max_depth = std::max(P.max_depth, H);
            const int fid = (int)P.fmm.size();
            F.nsrc = (int)S.size();
            F.ntgt = (int)T.size();
            int shH = kCellBits - H;
            // boxes per level, in Morton order (prefixes of the sorted fine keys)
            std::vector<BoxSet> SB(H + 1), TB(H + 1);
            auto make_boxes = [&](const std::vector<Pt>& V, std::vector<BoxSet>& B) {
                for (int lv = 0; lv <= H; ++lv) {
                    int sh = kCellBits - lv;
                    BoxSet& bs = B[lv];
                    for (size_t i = 0; i < V.size(); ++i) {
                        if (i > 0 && (V[i].fkey >> (3 * sh)) == (V[i - 1].fkey >> (3 * sh))) continue;
                        uint32_t a = V[i].c[0] >> sh, b = V[i].c[1] >> sh, c = V[i].c[2] >> sh;
                        bs.idx[cellkey(a, b, c)] = (int)bs.mkey.size();
                        bs.mkey.push_back(V[i].fkey >> (3 * sh));
                        bs.ix.push_back((int)a);
                        bs.iy.push_back((int)b);
                        bs.iz.push_back((int)c);
                    }
                }
            };
            make_boxes(S, SB);
            make_boxes(T, TB);
            // global ME / LE indices for levels >= 2
            for (int lv = 0; lv <= kMaxDepth; ++lv) {
                F.me_off[lv] = F.le_off[lv] = -1;
                F.me_cnt[lv] = F.le_cnt[lv] = 0;
            }
            for (int lv = 2; lv <= H; ++lv) {
                F.me_off[lv] = P.n_me;
                F.me_cnt[lv] = (int)SB[lv].mkey.size();
                for (int k = 0; k < F.me_cnt[lv]; ++k) { P.me_fmm.push_back(fid); P.me_level.push_back(lv); }
                P.n_me += F.me_cnt[lv];
                F.le_off[lv] = P.n_le;
                F.le_cnt[lv] = (int)TB[lv].mkey.size();
                for (int k = 0; k < F.le_cnt[lv]; ++k) { P.le_fmm.push_back(fid); P.le_level.push_back(lv); }
                P.n_le += F.le_cnt[lv];
            }
            m2l_by_le.resize(P.n_le);
            auto hlev = [&](int lv) { return 2.0 * F.R / (double)(1 << lv); };
            auto centre = [&](int lv, int i) { return -F.R + (i + 0.5) * hlev(lv); };   // canonical local frame
            // ---- points and leaves ----
            const int sl0 = (int)P.sl_me.size();
            {
                int cur = -1;
                for (size_t k = 0; k < S.size(); ++k) {
                    uint32_t a = S[k].c[0] >> shH, b = S[k].c[1] >> shH, c = S[k].c[2] >> shH;
                    int bi = SB[H].idx[cellkey(a, b, c)];
                    if (bi != cur) {
                        if (cur >= 0) P.sl_start.push_back((int)P.s_cidx.size());
                        cur = bi;
                        P.sl_me.push_back(H >= 2 ? F.me_off[H] + bi : -1);
                        P.sl_fmm.push_back(fid);
                        P.sl_level.push_back(H);
                        P.sl_h.push_back(hlev(H));
                        P.sl_ctr.push_back(centre(H, (int)a));
                        P.sl_ctr.push_back(centre(H, (int)b));
                        P.sl_ctr.push_back(centre(H, (int)c));
                    }
                    P.s_cidx.push_back(S[k].cidx);
                    P.s_okey.push_back(morton(a, b, F.flip < 0 ? (uint32_t)((1 << H) - 1) - c : c, H));
                    double zl = (double)F.flip * (S[k].z - F.cz);
                    s_ux.push_back((S[k].x - F.cx) - centre(H, (int)a));
                    s_uy.push_back((S[k].y - F.cy) - centre(H, (int)b));
                    s_uz.push_back(zl - centre(H, (int)c));
                }
                P.sl_start.push_back((int)P.s_cidx.size());
            }
            const int tl0 = (int)P.tl_le.size();
            {
                int cur = -1;
                for (size_t k = 0; k < T.size(); ++k) {
                    uint32_t a = T[k].c[0] >> shH, b = T[k].c[1] >> shH, c = T[k].c[2] >> shH;
                    int bi = TB[H].idx[cellkey(a, b, c)];
                    if (bi != cur) {
                        if (cur >= 0) P.tl_start.push_back((int)P.t_cidx.size());
                        cur = bi;
                        P.tl_le.push_back(H >= 2 ? F.le_off[H] + bi : -1);
                        P.tl_fmm.push_back(fid);
                        P.tl_h.push_back(hlev(H));
                        P.tl_ctr.push_back(centre(H, (int)a));
                        P.tl_ctr.push_back(centre(H, (int)b));
                        P.tl_ctr.push_back(centre(H, (int)c));
                    }
                    P.t_cidx.push_back(T[k].cidx);
                    P.t_okey.push_back(morton(a, b, F.flip < 0 ? (uint32_t)((1 << H) - 1) - c : c, H));
                    P.t_out.push_back(slot);   // finalised below with ncharges
                    double zl = (double)F.flip * (T[k].z - F.cz);
                    t_ux.push_back((T[k].x - F.cx) - centre(H, (int)a));
                    t_uy.push_back((T[k].y - F.cy) - centre(H, (int)b));
                    t_uz.push_back(zl - centre(H, (int)c));
                }
                P.tl_start.push_back((int)P.t_cidx.size());
            }
            // ---- operators: M2M (parent level lv, octant), L2L (child level lv, octant) ----
            int m2m_op[kMaxDepth + 1][8], l2l_op[kMaxDepth + 1][8];
            for (int lv = 2; lv < H; ++lv)
                for (int o = 0; o < 8; ++o) {
                    double hc = hlev(lv + 1);
                    OpDesc d{};
                    d.type = OP_M2M;
                    d.fmm = fid;
                    d.level = lv;
                    d.rkey = -1;
                    // b = child centre - parent centre
                    d.bx = (((o >> 2) & 1) - 0.5) * hc;
                    d.by = (((o >> 1) & 1) - 0.5) * hc;
                    d.bz = ((o & 1) - 0.5) * hc;
                    m2m_op[lv][o] = (int)P.ops.size();
                    P.ops.push_back(d);
                }
            for (int lv = 3; lv <= H; ++lv)
                for (int o = 0; o < 8; ++o) {
                    double hc = hlev(lv);
                    OpDesc d{};
                    d.type = OP_L2L;
                    d.fmm = fid;
                    d.level = lv;
                    d.rkey = -1;
                    d.bx = (((o >> 2) & 1) - 0.5) * hc;
                    d.by = (((o >> 1) & 1) - 0.5) * hc;
                    d.bz = ((o & 1) - 0.5) * hc;
                    l2l_op[lv][o] = (int)P.ops.size();
                    P.ops.push_back(d);
                }
            // M2M lists
            for (int lv = 2; lv < H; ++lv) {
                for (int k = 0; k < (int)SB[lv].mkey.size(); ++k) {
                    int px = SB[lv].ix[k], py = SB[lv].iy[k], pz = SB[lv].iz[k];
                    for (int o = 0; o < 8; ++o) {
                        int cx = 2 * px + ((o >> 2) & 1), cy = 2 * py + ((o >> 1) & 1), cz = 2 * pz + (o & 1);
                        auto it = SB[lv + 1].idx.find(cellkey(cx, cy, cz));
                        if (it == SB[lv + 1].idx.end()) continue;
                        m2m_by_level[lv].push_back({F.me_off[lv] + k, F.me_off[lv + 1] + it->second, m2m_op[lv][o]});
                    }
                }
            }
            // L2L lists
            for (int lv = 3; lv <= H; ++lv)
                for (int k = 0; k < (int)TB[lv].mkey.size(); ++k) {
                    int ix = TB[lv].ix[k], iy = TB[lv].iy[k], iz = TB[lv].iz[k];
                    int pk = TB[lv - 1].idx.at(cellkey(ix >> 1, iy >> 1, iz >> 1));
                    int o = ((ix & 1) << 2) | ((iy & 1) << 1) | (iz & 1);
                    l2l_by_level[lv].push_back({F.le_off[lv] + k, F.le_off[lv - 1] + pk, l2l_op[lv][o]});
                }
            // M2L (V-lists) with operator de-duplication
            std::unordered_map<uint64_t, int> opmap, rkmap;
            auto free_op = [&](int lv, int dx, int dy, int dz) {
                uint64_t key = ((uint64_t)lv << 16) | (uint64_t)(((dx + 3) * 7 + (dy + 3)) * 7 + (dz + 3));
                auto f = opmap.find(key);
                if (f != opmap.end()) return f->second;
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
                opmap[key] = op;
                return op;
            };
            // tiled levels of a free-space FMM: dense grids, operator table, tiles
            int tiled_max = (cp.kind == 0) ? std::min(H, kTileMaxLevel) : 1;
            for (int lv = 2; lv <= tiled_max; ++lv) {
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
                    P.grid_me[t.grid_off + ((size_t)SB[lv].ix[k] * nside + SB[lv].iy[k]) * nside + SB[lv].iz[k]] = F.me_off[lv] + k;
                for (int k = 0; k < (int)TB[lv].mkey.size(); ++k)
                    P.grid_le[t.grid_off + ((size_t)TB[lv].ix[k] * nside + TB[lv].iy[k]) * nside + TB[lv].iz[k]] = F.le_off[lv] + k;
                P.optab.resize(P.optab.size() + 343, -1);
                for (int dx = -3; dx <= 3; ++dx)
                    for (int dy = -3; dy <= 3; ++dy)
                        for (int dz = -3; dz <= 3; ++dz) {
                            if (std::abs(dx) <= 1 && std::abs(dy) <= 1 && std::abs(dz) <= 1) continue;
                            P.optab[t.optab_off + ((dx + 3) * 7 + (dy + 3)) * 7 + (dz + 3)] = free_op(lv, dx, dy, dz);
                        }
                int fl = (int)P.tfl.size();
                P.tfl.push_back(t);
                int np = nside / 2;
                for (int bx = 0; bx < np; bx += kTilePB)
                    for (int by = 0; by < np; by += kTilePB)
                        for (int bz = 0; bz < np; bz += kTilePB)
                            for (int o = 0; o < 8; ++o) {
                                bool any = false;
                                for (int i = 0; i < kTilePB && !any; ++i)
                                    for (int j = 0; j < kTilePB && !any; ++j)
                                        for (int k = 0; k < kTilePB && !any; ++k) {
                                            int tx = 2 * (bx + i) + ((o >> 2) & 1), ty = 2 * (by + j) + ((o >> 1) & 1),
                                                tz = 2 * (bz + k) + (o & 1);
                                            if (tx < nside && ty < nside && tz < nside &&
                                                P.grid_le[t.grid_off + ((size_t)tx * nside + ty) * nside + tz] >= 0)
                                                any = true;
                                        }
                                if (any) P.tiles.push_back({fl, o, bx, by, bz});
                            }
            }
            for (int lv = 2; lv <= H; ++lv) {
                const bool tiled = lv <= tiled_max;
                int nside = 1 << lv;
                double h = hlev(lv);
                for (int k = 0; k < (int)TB[lv].mkey.size(); ++k) {
                    int tx = TB[lv].ix[k], ty = TB[lv].iy[k], tz = TB[lv].iz[k];
                    int le = F.le_off[lv] + k;
                    for (int qx = (tx >> 1) - 1; qx <= (tx >> 1) + 1; ++qx)
                        for (int qy = (ty >> 1) - 1; qy <= (ty >> 1) + 1; ++qy)
                            for (int qz = (tz >> 1) - 1; qz <= (tz >> 1) + 1; ++qz) {
                                if (qx < 0 || qy < 0 || qz < 0 || qx >= nside / 2 || qy >= nside / 2 || qz >= nside / 2)
                                    continue;
                                for (int o = 0; o < 8; ++o) {
                                    int sx = 2 * qx + ((o >> 2) & 1), sy = 2 * qy + ((o >> 1) & 1), sz = 2 * qz + (o & 1);
                                    int dx = sx - tx, dy = sy - ty, dz = sz - tz;
                                    if (std::abs(dx) <= 1 && std::abs(dy) <= 1 && std::abs(dz) <= 1) continue;
                                    auto it = SB[lv].idx.find(cellkey(sx, sy, sz));
                                    if (it == SB[lv].idx.end()) continue;
                                    int op;
                                    if (cp.kind == 0) {
                                        op = free_op(lv, dx, dy, dz);
                                    } else {
                                        uint64_t key = ((uint64_t)lv << 48) | ((uint64_t)(dx + 3) << 40) | ((uint64_t)(dy + 3) << 32) |
                                                       ((uint64_t)tz << 16) | (uint64_t)sz;
                                        auto f = opmap.find(key);
                                        if (f == opmap.end()) {
                                            int d2 = dx * dx + dy * dy;
                                            uint64_t rk = ((uint64_t)lv << 48) | ((uint64_t)d2 << 32) | ((uint64_t)tz << 16) | (uint64_t)sz;
                                            int rki;
                                            auto g = rkmap.find(rk);
                                            if (g == rkmap.end()) {
                                                RKey r{};
                                                r.fmm = fid;
                                                r.level = lv;
                                                r.rho = h * std::sqrt((double)d2);
                                                r.zt = centre(lv, tz);
                                                r.zs = centre(lv, sz);
                                                r.S = h;
                                                rki = (int)P.rkeys.size();
                                                P.rkeys.push_back(r);
                                                rkmap[rk] = rki;
                                            } else rki = g->second;
                                            OpDesc d{};
                                            d.type = OP_M2L_REACT;
                                            d.fmm = fid;
                                            d.level = lv;
                                            d.rkey = rki;
                                            d.phi = (dx == 0 && dy == 0) ? 0.0 : std::atan2((double)-dy, (double)-dx);
                                            op = (int)P.ops.size();
                                            P.ops.push_back(d);
                                            opmap[key] = op;
                                        } else op = f->second;
                                    }
                                    if (!tiled) m2l_by_le[le].push_back({F.me_off[lv] + it->second, op});
                                    else P.n_m2l_tile_pairs++;
                                    P.n_m2l_pairs++;
                                }
                            }
                }
            }
            // U-lists at the leaf level
            {
                int nside = 1 << H;
                int ntl = (int)TB[H].mkey.size();
                // target leaf order equals TB[H] order (both sorted by Morton key)
                p2p_by_tl.resize(tl0 + ntl);
                for (int k = 0; k < ntl; ++k) {
                    int tx = TB[H].ix[k], ty = TB[H].iy[k], tz = TB[H].iz[k];
                    int nt = P.tl_start[tl0 + k + 1] - P.tl_start[tl0 + k];
                    for (int dx = -1; dx <= 1; ++dx)
                        for (int dy = -1; dy <= 1; ++dy)
                            for (int dz = -1; dz <= 1; ++dz) {
                                int sx = tx + dx, sy = ty + dy, sz = tz + dz;
                                if (sx < 0 || sy < 0 || sz < 0 || sx >= nside || sy >= nside || sz >= nside) continue;
                                auto it = SB[H].idx.find(cellkey(sx, sy, sz));
                                if (it == SB[H].idx.end()) continue;
                                int sl = sl0 + it->second;
                                p2p_by_tl[tl0 + k].push_back(sl);
                                int64_t pairs = (int64_t)nt * (P.sl_start[sl + 1] - P.sl_start[sl]);
                                P.n_p2p_pairs += pairs;
                                if (cp.kind == 1) P.n_react_p2p_pairs += pairs;
                            }
                }
            }
            P.fmm.push_back(F);
        }
    }
    // ---- finalise flattened arrays ----
    P.s_u.resize(3 * s_ux.size());
    for (size_t i = 0; i < s_ux.size(); ++i) {
        P.s_u[i] = s_ux[i];
        P.s_u[s_ux.size() + i] = s_uy[i];
        P.s_u[2 * s_ux.size() + i] = s_uz[i];
    }
    P.t_u.resize(3 * t_ux.size());
    for (size_t i = 0; i < t_ux.size(); ++i) {
        P.t_u[i] = t_ux[i];
        P.t_u[t_ux.size() + i] = t_uy[i];
        P.t_u[2 * t_ux.size() + i] = t_uz[i];
    }
    for (size_t i = 0; i < P.t_out.size(); ++i) P.t_out[i] = (int)(P.t_out[i] * P.ncharges + P.t_cidx[i]);
    P.m2m_parent.clear(); P.m2m_ptr.assign(1, 0); P.m2m_child.clear(); P.m2m_op.clear();
    P.m2m_level_ptr.assign(kMaxDepth + 2, 0);
    for (int lv = 0; lv <= kMaxDepth; ++lv) {
        P.m2m_level_ptr[lv] = (int)P.m2m_parent.size();
        auto& v = m2m_by_level[lv];
        std::stable_sort(v.begin(), v.end(), [](const M2MRec& a, const M2MRec& b) { return a.parent < b.parent; });
        for (size_t i = 0; i < v.size(); ++i) {
            if (i == 0 || v[i].parent != v[i - 1].parent) {
                if (i > 0) P.m2m_ptr.push_back((int)P.m2m_child.size());
                P.m2m_parent.push_back(v[i].parent);
            }
            P.m2m_child.push_back(v[i].child);
            P.m2m_op.push_back(v[i].op);
        }
        if (!v.empty()) P.m2m_ptr.push_back((int)P.m2m_child.size());
    }
    P.m2m_level_ptr[kMaxDepth + 1] = (int)P.m2m_parent.size();
    P.l2l_child.clear(); P.l2l_parent.clear(); P.l2l_op.clear();
    P.l2l_level_ptr.assign(kMaxDepth + 2, 0);
    for (int lv = 0; lv <= kMaxDepth; ++lv) {
        P.l2l_level_ptr[lv] = (int)P.l2l_child.size();
        for (auto& r : l2l_by_level[lv]) {
            P.l2l_child.push_back(r.child);
            P.l2l_parent.push_back(r.parent);
            P.l2l_op.push_back(r.op);
        }
    }
    P.l2l_level_ptr[kMaxDepth + 1] = (int)P.l2l_child.size();
    P.m2l_ptr.assign(1, 0); P.m2l_src.clear(); P.m2l_op.clear();
    m2l_by_le.resize(P.n_le);
    for (int i = 0; i < P.n_le; ++i) {
        for (auto& e : m2l_by_le[i]) {
            P.m2l_src.push_back(e.first);
            P.m2l_op.push_back(e.second);
        }
        P.m2l_ptr.push_back((int)P.m2l_src.size());
    }
    P.swz_ops.clear();
    P.swz_index.assign(P.ops.size(), -1);
    for (size_t i = 0; i < P.ops.size(); ++i)
        if (P.ops[i].type == OP_M2L_FREE) {
            P.swz_index[i] = (int)P.swz_ops.size();
            P.swz_ops.push_back((int)i);
        }
    P.p2p_ptr.assign(1, 0); P.p2p_src.clear();
    p2p_by_tl.resize(P.tl_le.size());
    for (auto& v : p2p_by_tl) {
        for (int sl : v) P.p2p_src.push_back(sl);
        P.p2p_ptr.push_back((int)P.p2p_src.size());
    }
    (void)p;
    return "";
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
