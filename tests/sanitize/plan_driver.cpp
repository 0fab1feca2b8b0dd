// Sanitizer driver for the host plan builder (test infrastructure; built with
// AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_sanitizers.py).
// A host stand-in of the point builder (the device builder's rules: fine
// cells, stable key sort, uniform and adaptive leaves) feeds build_plan on
// uniform, clustered and interface-clustered inputs, uniform and adaptive
// trees; every index the plan hands to the kernels is checked against its
// array.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <functional>
#include <random>

#include "../../paper_2002_01334_amd/csrc/lpb_internal.h"

using namespace lpb;

namespace {

uint32_t fine(double w, double R)
{
    double f = std::floor((w + R) / (2.0 * R) * 65536.0);
    if (!(f >= 0.0)) f = 0.0;
    if (f > 65535.0) f = 65535.0;
    return (uint32_t)f;
}

struct HostPB : PointBuilder {
    const std::vector<std::vector<double>>*xs, *ys, *zs;
    std::vector<std::vector<uint64_t>> K;
    int keys(int sys, int64_t, const std::vector<int>& mem, const SetFrame& F, double R, int counts[kMaxDepth + 1],
             std::string&) override
    {
        std::vector<std::pair<uint64_t, int>> v(mem.size());
        for (size_t i = 0; i < mem.size(); ++i) {
            const int m = mem[i];
            const double w0 = (*xs)[sys][m] - F.ax, w1 = (*ys)[sys][m] - F.ay, z = (*zs)[sys][m];
            double w2;
            if (F.mode == 0) w2 = z - F.az;
            else {
                const double t = F.side == 1 ? z - F.az : F.az - z;
                w2 = F.target ? t : -t;
            }
            v[i] = {(morton_spread3(fine(w0, R)) << 2) | (morton_spread3(fine(w1, R)) << 1) | morton_spread3(fine(w2, R)),
                    (int)i};
        }
        std::stable_sort(v.begin(), v.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
        std::vector<uint64_t> k(v.size());
        for (size_t i = 0; i < v.size(); ++i) k[i] = v[i].first;
        for (int lv = 0; lv <= kMaxDepth; ++lv) {
            const int sh = 3 * (kCellBits - lv);
            int n = 0;
            for (size_t i = 0; i < k.size(); ++i) n += (i == 0 || (k[i] >> sh) != (k[i - 1] >> sh));
            counts[lv] = n;
        }
        K.push_back(std::move(k));
        return (int)K.size() - 1;
    }
    bool leaves(int h, int H, std::vector<uint64_t>& lk, std::vector<int>& ls, std::string&) override
    {
        const auto& k = K[h];
        const int sh = 3 * (kCellBits - H);
        lk.clear();
        ls.clear();
        for (size_t i = 0; i < k.size(); ++i)
            if (i == 0 || (k[i] >> sh) != (k[i - 1] >> sh)) {
                lk.push_back(k[i] >> sh);
                ls.push_back((int)i);
            }
        return true;
    }
    bool leaves_adaptive(int h, int cap, bool sep, std::vector<uint64_t>& lk, std::vector<int>& llv,
                         std::vector<int>& ls, std::string&) override
    {
        const auto& k = K[h];
        lk.clear();
        llv.clear();
        ls.clear();
        const int n = (int)k.size();
        if (!n) return true;
        std::function<void(int, int, int, int)> divide = [&](int a, int b, int lv, int locc) {
            bool split = false;
            if (lv < kMaxDepth) {
                if (b - a > cap) {
                    split = true;
                    locc = -1;
                } else {
                    if (locc < 0) locc = lv;
                    if (sep && lv < locc + 3) {
                        uint32_t dmin = 0xffffffffu;
                        for (int i = a; i < b; ++i) {
                            const uint32_t cz = morton_compact3(k[i]);
                            dmin = std::min(dmin, cz >= 32768u ? cz - 32768u : 32767u - cz);
                        }
                        split = (1u << (kCellBits - lv)) > dmin;
                    }
                }
            }
            if (!split) {
                lk.push_back(k[a] >> (3 * (kCellBits - lv)));
                llv.push_back(lv);
                ls.push_back(a);
                return;
            }
            const int sh = 3 * (kCellBits - lv - 1);
            for (int c = a; c < b;) {
                const uint64_t last = (((k[c] >> sh) + 1) << sh) - 1;
                const int e = (int)(std::upper_bound(k.begin() + c, k.begin() + b, last) - k.begin());
                divide(c, e, lv + 1, locc);
                c = e;
            }
        };
        divide(0, n, 0, -1);
        return true;
    }
    int failure() const override { return LPB_EDEVICE; }
};

int fails = 0;
void expect(bool ok, const char* what, int a = 0)
{
    if (!ok && fails++ < 20) std::fprintf(stderr, "FAIL %s (%d)\n", what, a);
}

template <typename V>
void check_csr(const std::vector<int>& ptr, const std::vector<V>& idx, size_t nrows, int64_t lim, const char* what)
{
    expect(ptr.size() == nrows + 1, what);
    for (size_t i = 0; i + 1 < ptr.size(); ++i) expect(ptr[i] <= ptr[i + 1], what);
    if (!ptr.empty()) expect(ptr.front() == 0 && (size_t)ptr.back() == idx.size(), what);
    for (auto v : idx) expect(v >= 0 && (int64_t)v < lim, what, (int)v);
}

void check_plan(const Plan& P)
{
    const size_t ns = P.sl_me.size(), nt = P.tl_le.size();
    expect(P.sl_start.size() == ns + 1 && P.tl_start.size() == nt + 1, "leaf starts");
    for (size_t i = 0; i < ns; ++i) expect(P.sl_start[i] < P.sl_start[i + 1] && P.sl_me[i] < P.n_me, "source leaf");
    for (size_t i = 0; i < nt; ++i) expect(P.tl_start[i] < P.tl_start[i + 1] && P.tl_le[i] < P.n_le, "target leaf");
    if (ns) expect(P.sl_start[ns] == P.n_spts, "source points");
    if (nt) expect(P.tl_start[nt] == P.n_tpts, "target points");
    expect(P.sl_lv.size() == ns && P.tl_lv.size() == nt, "leaf levels");
    check_csr(P.m2l_ptr, P.m2l_src, (size_t)P.n_le, P.n_me, "m2l");
    for (int op : P.m2l_op) expect(op >= 0 && op < (int)P.ops.size(), "m2l op");
    check_csr(P.p2p_ptr, P.p2p_src, nt, (int64_t)ns, "p2p");
    check_csr(P.rp_ptr, P.rp_src, nt, (int64_t)ns, "rp");
    for (int f : P.rp_fmm) expect(f >= 0 && f < (int)P.fmm.size(), "rp fmm");
    check_csr(P.w_ptr, P.w_me, nt, P.n_me, "w");
    for (size_t e = 0; e < P.w_fmm.size(); ++e) expect(P.w_lv[e] >= 2 && P.w_lv[e] <= kMaxDepth, "w level");
    check_csr(P.x_box_ptr, P.x_sl, P.x_box_le.size(), (int64_t)ns, "x");
    for (int le : P.x_box_le) expect(le >= 0 && le < P.n_le, "x box");
    for (size_t t = 0; t + 1 < P.bw_term_ptr.size(); ++t) expect(P.bw_term_ptr[t] <= P.bw_term_ptr[t + 1], "bw terms");
    for (int v : P.bw_op) expect(v >= 0 && v < (int)P.ops.size(), "bw op");
    for (int v : P.bw_src) expect(v >= -1, "bw src");
    int64_t vec = 0;
    for (const auto& o : P.pt_ops) {
        expect(o.out == vec, "point op offset");
        vec += P.K;
        expect(o.kind == 0 ? (o.pt >= 0 && o.pt < P.n_tpts && o.leaf >= 0 && o.leaf < (int)nt)
                           : (o.pt >= 0 && o.pt < P.n_spts && o.leaf >= 0 && o.leaf < (int)ns),
               "point op point");
    }
    for (const auto& t : P.tiles) expect(t.fl >= 0 && t.fl < (int)P.tfl.size(), "tile");
}

}  // namespace

int main()
{
    std::mt19937_64 g(17);
    std::uniform_real_distribution<double> u(0.0, 1.0);
    std::normal_distribution<double> nd(0.0, 1.0);
    Medium M3{};
    M3.L = 2;
    const double eps[3] = {1, 2, 4}, lam[3] = {1.2, 1.5, 2.0};
    for (int l = 0; l < 3; ++l) {
        M3.eps[l] = eps[l];
        M3.lam[l] = lam[l];
    }
    M3.d[0] = 0.0;
    M3.d[1] = -1.2;
    Medium M1{};
    M1.L = 0;
    M1.eps[0] = 2.0;
    M1.lam[0] = 0.8;
    const double slab[3][2] = {{0.01, 1.0}, {-1.19, -0.01}, {-2.2, -1.21}};
    const double cz[3] = {0.04, -0.04, -1.24};
    int cases = 0;
    for (int recipe = 0; recipe < 3; ++recipe) {
        const bool layered = recipe != 2;
        std::vector<std::vector<double>> xs(1), ys(1), zs(1);
        const int per = 700;
        for (int l = 0; l < (layered ? 3 : 1); ++l)
            for (int i = 0; i < per; ++i) {
                double x, y, z;
                if (recipe == 0 || i % 2) {
                    x = u(g) - 0.5;
                    y = u(g) - 0.5;
                    z = layered ? slab[l][0] + (slab[l][1] - slab[l][0]) * u(g) : u(g) - 0.5;
                } else {
                    do {
                        x = 0.1 + 0.03 * nd(g);
                        y = -0.1 + 0.03 * nd(g);
                        z = (layered ? cz[l] : 0.2) + 0.01 * nd(g);
                    } while (x < -0.5 || x > 0.5 || y < -0.5 || y > 0.5 ||
                             (layered && (z < slab[l][0] || z > slab[l][1])));
                }
                xs[0].push_back(x);
                ys[0].push_back(y);
                zs[0].push_back(z);
            }
        for (int mode = 0; mode <= 2; ++mode)
            for (int cap : {3, 20, 60}) {
                Plan P;
                P.p = 5;
                P.K = 36;
                P.leaf_cap = cap;
                P.adaptive = mode;
                HostPB pb;
                pb.xs = &xs;
                pb.ys = &ys;
                pb.zs = &zs;
                int st = 0;
                const std::string msg = build_plan(P, {layered ? M3 : M1}, xs, ys, zs, 1e-9, pb, &st);
                expect(msg.empty() && st == 0, "build_plan", recipe * 100 + mode * 10);
                check_plan(P);
                ++cases;
            }
    }
    std::printf("plans checked: %d, failures: %d\n", cases, fails);
    return fails ? 1 : 0;
}
