// lpb_capi.cpp -- the C ABI of include/lpb.h: context, validation, device
// memory, plan upload, operator generation and evaluation on the stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "lpb_eval.h"
#include "lpb_tree_dev.h"
#include "lpb_internal.h"
#include "lpb_opgen.h"

using namespace lpb;

// Partial potentials of lpb_evaluate_noalloc: one array per GPU, held until
// the process ends.  Host code never passes this name to a kernel (on the
// host it only stands for the symbol): the device address of each GPU's copy
// comes from hipGetSymbolAddress, looked up once per device in lpb_create.
static __device__ __align__(256) double scratch[LPB_NOALLOC_MAX_PARTS];

namespace {

thread_local std::string g_create_error;

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (which must be current), looked
// up on the first call for that device.
hipError_t scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = (double*)ptr;
    return hipSuccess;
}

double* scratch_ptr(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}

struct DevBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
};

}  // namespace

struct lpb_ctx {
    lpb_options opt{};
    hipStream_t stream = nullptr;
    std::string err;
    // problem
    bool have_layers = false, have_tree = false, batched = false;
    std::vector<Medium> media;
    std::vector<std::vector<double>> xs, ys, zs;
    Plan plan;
    bool ops_dirty = true;
    // host tables (depend on p only)
    std::vector<double> btab, gtab;
    // device memory
    std::vector<DevBuf> plan_bufs;   // freed on every plan rebuild
    std::vector<DevBuf> op_bufs;     // freed on every operator rebuild
    DevBuf d_btab, d_gtab, d_glx, d_glw, d_flag;
    double* d_q = nullptr;
    double* d_phi = nullptr;
    void* d_pool_eval = nullptr;
    // kernel arguments
    EvalArgs<double> a64{};
    EvalArgs<float> a32{};
    EvalSched sched{};
    OpgenInputs og{};
    lpb_stats stats{};
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipEvent_t evs[11] = {};
    // captured evaluation passes (options.graph)
    hipStream_t own_stream = nullptr;   // capture needs a stream other than the null stream
    EvalFork fork{};                    // side stream (default priority) and its events
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    bool tune_needed = true;
    bool prepared = false;   // lpb_evaluate has run since the last plan or operator change
};

namespace {

void drop_graph(lpb_ctx* c)
{
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
}

lpb_status fail(lpb_ctx* c, lpb_status s, const std::string& msg)
{
    if (c) c->err = msg;
    else g_create_error = msg;
    return s;
}

#define HIPCHK(c, call)                                                                              \
    do {                                                                                             \
        hipError_t e_ = (call);                                                                      \
        if (e_ != hipSuccess)                                                                        \
            return fail((c), e_ == hipErrorOutOfMemory ? LPB_ENOMEM : LPB_EDEVICE,                   \
                        std::string(#call) + ": " + hipGetErrorString(e_));                          \
    } while (0)

// Device memory of a context: the caller's allocator hook when set, else
// hipMalloc / hipFree.  Buffers are only returned after the context's stream
// has drained (no kernel still reads them).
void* dev_alloc(lpb_ctx* c, size_t bytes)
{
    if (c->opt.alloc) return c->opt.alloc(bytes, c->opt.alloc_user);
    void* p = nullptr;
    return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
}

void dev_free(lpb_ctx* c, void* p)
{
    if (!p) return;
    if (c->opt.alloc) c->opt.free(p, c->opt.alloc_user);
    else (void)hipFree(p);
}

void free_buf(lpb_ctx* c, DevBuf& b)
{
    dev_free(c, b.ptr);
    b.ptr = nullptr;
    b.bytes = 0;
}

void free_bufs(lpb_ctx* c, std::vector<DevBuf>& v)
{
    if (!v.empty()) (void)hipStreamSynchronize(c->stream);
    for (auto& b : v) free_buf(c, b);
    v.clear();
}

template <typename T>
lpb_status dalloc(lpb_ctx* c, std::vector<DevBuf>& pool, size_t n, T** out)
{
    *out = nullptr;
    size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
    void* p = dev_alloc(c, bytes);
    if (!p) return fail(c, LPB_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    pool.push_back({p, bytes});
    *out = (T*)p;
    return LPB_OK;
}

template <typename T>
lpb_status upload(lpb_ctx* c, std::vector<DevBuf>& pool, const std::vector<T>& v, T** out)
{
    lpb_status s = dalloc<T>(c, pool, v.size(), out);
    if (s != LPB_OK) return s;
    if (!v.empty()) {
        hipError_t e = hipMemcpy(*out, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
        if (e != hipSuccess) return fail(c, LPB_EDEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
    }
    return LPB_OK;
}

// b^t_{nm} of the Legendre-product expansion (Sec. 3.5):
//   a^j_{nm} = (-1)^{n-j} (2j)! c_nm / (2^n j! (n-j)! (2j-n-m)!),
//   b^t_{nm} = sum_{j=q}^{n} (-1)^t a^j_{nm} (j-r)! / (t! (j-r-t)!),
//   r = floor((n+m)/2), q = max(ceil((n+m)/2), t+r),  c_nm = sqrt((2n+1)/(4 pi) (n-m)!/(n+m)!).
void make_btab(int p, std::vector<double>& b)
{
    auto f = [](int n) {
        long double v = 1.0L;
        for (int k = 2; k <= n; ++k) v *= k;
        return v;
    };
    const int BT = p + 1;
    b.assign((size_t)(p + 1) * (p + 2) / 2 * BT, 0.0);
    for (int n = 0; n <= p; ++n)
        for (int m = 0; m <= n; ++m) {
            long double c = std::sqrt((2.0L * n + 1.0L) / (4.0L * 3.14159265358979323846264338327950288L) * f(n - m) / f(n + m));
            int r = (n + m) / 2;
            for (int t = 0; t <= n - r; ++t) {
                int q = std::max((n + m + 1) / 2, t + r);
                long double acc = 0.0L;
                for (int j = q; j <= n; ++j) {
                    long double a = (((n - j) & 1) ? -1.0L : 1.0L) * f(2 * j) * c /
                                    (std::pow(2.0L, n) * f(j) * f(n - j) * f(2 * j - n - m));
                    acc += ((t & 1) ? -1.0L : 1.0L) * a * f(j - r) / (f(t) * f(j - r - t));
                }
                b[(size_t)(n * (n + 1) / 2 + m) * BT + t] = (double)acc;
            }
        }
}

// G(n,m;nu,mu;q) = int Y_n^m conj(Y_nu^mu) conj(Y_q^{m-mu}) = (-1)^m gaunt(n,m; nu,-mu; q,mu-m)
void make_gtab(int p, std::vector<double>& g)
{
    const int K = (p + 1) * (p + 1), Kp = (p + 1) * (p + 2) / 2, NQ = 2 * p + 1;
    g.assign((size_t)Kp * K * NQ, 0.0);
    for (int n = 0; n <= p; ++n)
        for (int m = 0; m <= n; ++m)
            for (int nu = 0; nu <= p; ++nu)
                for (int mu = -nu; mu <= nu; ++mu)
                    for (int q = std::abs(n - nu); q <= n + nu; q += 2) {
                        if (std::abs(m - mu) > q) continue;
                        double v = ((m & 1) ? -1.0 : 1.0) * host_gaunt(n, m, nu, -mu, q, mu - m);
                        g[((size_t)(n * (n + 1) / 2 + m) * K + (nu * nu + nu + mu)) * NQ + q] = v;
                    }
}

lpb_status build_and_upload(lpb_ctx* c);

lpb_status check_layers(lpb_ctx* c, int nl, const double* eps, const double* lam, const double* d, Medium& M)
{
    if (nl < 1 || nl > LPB_MAX_LAYERS || nl - 1 > LPB_MAXL) return fail(c, LPB_EINVAL, "n_layers out of range");
    if (!eps || !lam || (nl > 1 && !d)) return fail(c, LPB_EINVAL, "null layer array");
    M = Medium{};
    M.L = nl - 1;
    for (int k = 0; k < nl; ++k) {
        if (!std::isfinite(eps[k]) || !std::isfinite(lam[k])) return fail(c, LPB_ENUMERIC, "non-finite eps/lambda");
        if (eps[k] <= 0.0 || lam[k] <= 0.0) return fail(c, LPB_EINVAL, "eps and lambda must be > 0");
        M.eps[k] = eps[k];
        M.lam[k] = lam[k];
    }
    for (int k = 0; k + 1 < nl; ++k) {
        if (!std::isfinite(d[k])) return fail(c, LPB_ENUMERIC, "non-finite interface");
        if (k > 0 && !(d[k] < d[k - 1])) return fail(c, LPB_EINVAL, "interfaces must be strictly decreasing");
        M.d[k] = d[k];
    }
    return LPB_OK;
}

lpb_status read_coords(lpb_ctx* c, int64_t n, const double* x, const double* y, const double* z, int on_device,
                       std::vector<double>& X, std::vector<double>& Y, std::vector<double>& Z)
{
    if (n < 0) return fail(c, LPB_EINVAL, "negative n");
    if (n > 0 && (!x || !y || !z)) return fail(c, LPB_EINVAL, "null coordinate array");
    X.resize(n);
    Y.resize(n);
    Z.resize(n);
    if (n == 0) return LPB_OK;
    if (on_device) {
        HIPCHK(c, hipMemcpy(X.data(), x, n * sizeof(double), hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(Y.data(), y, n * sizeof(double), hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(Z.data(), z, n * sizeof(double), hipMemcpyDeviceToHost));
    } else {
        std::memcpy(X.data(), x, n * sizeof(double));
        std::memcpy(Y.data(), y, n * sizeof(double));
        std::memcpy(Z.data(), z, n * sizeof(double));
    }
    return LPB_OK;
}

template <typename F, typename V>
lpb_status up_field(lpb_ctx* c, const F*& field, const std::vector<V>& vec)
{
    V* tmp = nullptr;
    lpb_status s = upload(c, c->plan_bufs, vec, &tmp);
    field = tmp;
    return s;
}


// Coefficients in sign-class order (natural order within a class), each
// class padded with -1 entries to a multiple of 16.
std::vector<int> class_rowmap(int p)
{
    std::vector<int> r;
    for (int cl = 0; cl < 8; ++cl) {
        for (int n = 0; n <= p; ++n)
            for (int m = 0; m <= n; ++m) {
                if (coef_class(n, m, 0) == cl) r.push_back(ire(n, m));
                if (m > 0 && coef_class(n, m, 1) == cl) r.push_back(iim(n, m));
            }
        while (r.size() % 16) r.push_back(-1);
    }
    return r;
}

template <typename T>
lpb_status fill_args(lpb_ctx* c, EvalArgs<T>& A, DevPointBuilder& pb)
{
    Plan& P = c->plan;
    lpb_status s;
    A = EvalArgs<T>{};
    A.p = P.p;
    A.K = P.K;
    A.KP = (P.K + 15) / 16 * 16;
    // the component slots, then the free-space near field's slot (added to
    // slot 0 by the final sum)
    A.nslots = P.nslots + 1;
    A.ncharges = P.ncharges;
    A.near_off = (int64_t)P.nslots * P.ncharges;
    A.n_src = (int)P.n_spts;
    A.quad_tol = c->opt.quad_tol;
    // FMM records
    std::vector<FmmDev> fd(P.fmm.size());
    for (size_t i = 0; i < P.fmm.size(); ++i) {
        const FmmDesc& F = P.fmm[i];
        FmmDev& D = fd[i];
        D.kind = F.kind; D.H = F.H; D.flip = F.flip; D.medium = F.sys;
        D.l = F.l; D.lp = F.lp; D.a = F.a; D.b = F.b;
        D.R = F.R; D.lam_s = F.lam_s; D.lam_t = F.lam_t; D.far_factor = F.far_factor; D.eps_t = F.eps_t;
        for (int l = 0; l <= kMaxDepth; ++l) { D.me_off[l] = F.me_off[l]; D.le_off[l] = F.le_off[l]; }
    }
    FmmDev* dfmm;
    Medium* dmed;
    if ((s = upload(c, c->plan_bufs, fd, &dfmm)) != LPB_OK) return s;
    if ((s = upload(c, c->plan_bufs, P.media, &dmed)) != LPB_OK) return s;
    A.fmm = dfmm;
    A.media = dmed;
#define UP(field, vec)                                                     \
    if ((s = up_field(c, A.field, vec)) != LPB_OK) return s;
    UP(sl_start, P.sl_start);
    UP(sl_me, P.sl_me);
    UP(sl_fmm, P.sl_fmm);
    UP(sl_h, P.sl_h);
    UP(sl_ctr, P.sl_ctr);
    UP(tl_start, P.tl_start);
    UP(tl_le, P.tl_le);
    UP(tl_fmm, P.tl_fmm);
    UP(tl_h, P.tl_h);
    UP(tl_ctr, P.tl_ctr);
    UP(sl_lv, P.sl_lv);
    UP(tl_lv, P.tl_lv);
    {
        // adaptive trees: W-list (M2P) per target leaf, X-list (P2L) per target box
        std::vector<int> wl;
        for (size_t i = 0; i + 1 < P.w_ptr.size(); ++i)
            if (P.w_ptr[i + 1] > P.w_ptr[i]) wl.push_back((int)i);
        UP(w_leaves, wl);
        A.n_w_leaves = (int)wl.size();
        A.n_x_boxes = (int)P.x_box_le.size();
    }
    UP(w_ptr, P.w_ptr);
    UP(w_fmm, P.w_fmm);
    UP(w_me, P.w_me);
    UP(w_lv, P.w_lv);
    UP(w_ctr, P.w_ctr);
    UP(w_vec, P.w_vec);
    UP(x_box_le, P.x_box_le);
    UP(x_box_lv, P.x_box_lv);
    UP(x_box_ptr, P.x_box_ptr);
    UP(x_box_ctr, P.x_box_ctr);
    UP(x_fmm, P.x_fmm);
    UP(x_sl, P.x_sl);
    UP(x_vec, P.x_vec);
    UP(bw_term_ptr, P.bw_term_ptr);
    UP(bw_op, P.bw_op);
    UP(bw_src, P.bw_src);
    UP(bw_dst, P.bw_dst);
    UP(bw_xc, P.bw_xc);
    // cos and sin (m phi), m = 0..p, of the kXfDirs V-list directions:
    // e^{i phi} = (-dx - i dy) / |(dx, dy)| (phi = 0 for dx = dy = 0), powers in long double
    std::vector<T> rt((size_t)kXfDirs * (P.p + 1) * 2);
    {
        for (int dir = 0; dir < kXfDirs; ++dir) {
            const long double dx = dir / 7 - 3, dy = dir % 7 - 3, r = std::sqrt(dx * dx + dy * dy);
            const long double c1 = r > 0 ? -dx / r : 1.0L, s1 = r > 0 ? -dy / r : 0.0L;
            long double c = 1.0L, sn = 0.0L;
            for (int m = 0; m <= P.p; ++m) {
                rt[((size_t)dir * (P.p + 1) + m) * 2] = (T)c;
                rt[((size_t)dir * (P.p + 1) + m) * 2 + 1] = (T)sn;
                const long double c2 = c * c1 - sn * s1;
                sn = sn * c1 + c * s1;
                c = c2;
            }
        }
        UP(rot_tab, rt);
    }
    UP(m2l_ptr, P.m2l_ptr);
    UP(m2l_src, P.m2l_src);
    UP(m2l_op, P.m2l_op);
    UP(m2l_xc, P.m2l_xc);
    UP(p2p_ptr, P.p2p_ptr);
    UP(p2p_src, P.p2p_src);
    UP(rp_ptr, P.rp_ptr);
    UP(rp_fmm, P.rp_fmm);
    UP(rp_src, P.rp_src);
    UP(tiles, P.tiles);
    UP(tfl, P.tfl);
    UP(grid_me, P.grid_me);
    UP(grid_le, P.grid_le);
    UP(optab, P.optab);
    {
        // signs of the real-form coefficients under x -> -x (Re (-1)^m, Im -(-1)^m),
        // y -> -y (Re +1, Im -1) and z -> -z ((-1)^(n+m)); code bits 1 x, 2 y, 4 z
        std::vector<T> sg((size_t)8 * A.KP, T(1));
        for (int code = 0; code < 8; ++code)
            for (int n = 0; n <= P.p; ++n)
                for (int m = 0; m <= n; ++m) {
                    double re = 1.0, im = 1.0;
                    if (code & 1) { re *= (m & 1) ? -1.0 : 1.0; im *= (m & 1) ? 1.0 : -1.0; }
                    if (code & 2) im = -im;
                    if (code & 4) { double z = ((n + m) & 1) ? -1.0 : 1.0; re *= z; im *= z; }
                    sg[(size_t)code * A.KP + ire(n, m)] = (T)re;
                    if (m > 0) sg[(size_t)code * A.KP + iim(n, m)] = (T)im;
                }
        UP(refl_sign, sg);
        // the same transforms per (code, row) as one multiply-add,
        // row' = a row + b partner row: reflections (sign, 0), rotations
        // (1, 0) at m = 0, else (cos, sin) on Re rows, (cos, -sin) on Im rows
        std::vector<T> ab((size_t)(kXfRotate + kXfDirs) * P.K * 2, T(0));
        for (int code = 0; code < kXfRotate + kXfDirs; ++code)
            for (int n = 0; n <= P.p; ++n)
                for (int m = 0; m <= n; ++m) {
                    T* re = &ab[((size_t)code * P.K + ire(n, m)) * 2];
                    T* im = m > 0 ? &ab[((size_t)code * P.K + iim(n, m)) * 2] : nullptr;
                    if (code < kXfRotate) {
                        re[0] = sg[(size_t)code * A.KP + ire(n, m)];
                        if (im) im[0] = sg[(size_t)code * A.KP + iim(n, m)];
                    } else if (m == 0) {
                        re[0] = T(1);
                    } else {
                        const T* r = &rt[((size_t)(code - kXfRotate) * (P.p + 1) + m) * 2];
                        re[0] = r[0]; re[1] = r[1];
                        im[0] = r[0]; im[1] = -r[1];
                    }
                }
        UP(xf_ab, ab);
    }
    UP(oct_codes, P.oct_codes);
    UP(swz_index, P.swz_index);
    UP(orb_tab, P.orb_tab);
    UP(orb_index, P.orb_index);
    UP(orb_rows, class_rowmap(P.p));
    {
        std::vector<int> kc(A.KP, 0);
        for (int n = 0; n <= P.p; ++n)
            for (int m = 0; m <= n; ++m) {
                kc[ire(n, m)] = coef_class(n, m, 0);
                if (m > 0) kc[iim(n, m)] = coef_class(n, m, 1);
            }
        UP(orb_kcls, kc);
    }
    {
        // solid-harmonic recurrence tables (see lpb_math.h)
        std::vector<T> amm(P.p + 1), al((P.p + 1) * (P.p + 2) / 2, T(0)), be((P.p + 1) * (P.p + 2) / 2, T(0));
        double a = 0.28209479177387814;
        for (int m = 0; m <= P.p; ++m) {
            if (m > 0) a *= std::sqrt((2.0 * m + 1.0) / (2.0 * m));
            amm[m] = (T)a;
            if (m + 1 <= P.p) al[ipk(m + 1, m)] = (T)std::sqrt(2.0 * m + 3.0);
            for (int n = m + 2; n <= P.p; ++n) {
                double nn = (double)n * n, mm = (double)m * m;
                al[ipk(n, m)] = (T)std::sqrt((4.0 * nn - 1.0) / (nn - mm));
                be[ipk(n, m)] = (T)std::sqrt(((n - 1.0) * (n - 1.0) - mm) * (2.0 * n + 1.0) / ((nn - mm) * (2.0 * n - 3.0)));
            }
        }
        UP(sh_amm, amm);
        UP(sh_alpha, al);
        UP(sh_beta, be);
        const int Kp = (P.p + 1) * (P.p + 2) / 2;
        std::vector<double> s64((size_t)P.p + 1 + 2 * Kp, 0.0);
        double a64 = 0.28209479177387814;
        for (int m = 0; m <= P.p; ++m) {
            if (m > 0) a64 *= std::sqrt((2.0 * m + 1.0) / (2.0 * m));
            s64[m] = a64;
            if (m + 1 <= P.p) s64[P.p + 1 + ipk(m + 1, m)] = std::sqrt(2.0 * m + 3.0);
            for (int n = m + 2; n <= P.p; ++n) {
                double nn = (double)n * n, mm = (double)m * m;
                s64[P.p + 1 + ipk(n, m)] = std::sqrt((4.0 * nn - 1.0) / (nn - mm));
                s64[P.p + 1 + Kp + ipk(n, m)] =
                    std::sqrt(((n - 1.0) * (n - 1.0) - mm) * (2.0 * n + 1.0) / ((nn - mm) * (2.0 * n - 3.0)));
            }
        }
        UP(sh64, s64);
    }
    {
        // Bessel-ratio tables: factors of the it_n recurrence and series (p only) and
        // 1/it_n(lam h) for every FMM and level, source and target lambda
        const int NSER = 40, S0 = LPB_MAX_P + 2, S1 = S0 + NSER + 1;
        std::vector<double> tb(S1 + NSER + 1, 0.0);
        for (int n = 0; n <= P.p + 1; ++n) tb[n] = 1.0 / ((2.0 * n + 1.0) * (2.0 * n + 3.0));
        for (int k = 1; k <= NSER; ++k) {
            tb[S0 + k] = 1.0 / (2.0 * k * (2.0 * P.p + 2.0 * k + 1.0));
            tb[S1 + k] = 1.0 / (2.0 * k * (2.0 * (P.p + 1) + 2.0 * k + 1.0));
        }
        const size_t per = (size_t)(kMaxDepth + 1) * (LPB_MAX_P + 1);
        std::vector<double> is(P.fmm.size() * per, 1.0), it(P.fmm.size() * per, 1.0);
        double buf[LPB_MAX_P + 2];
        for (size_t f = 0; f < P.fmm.size(); ++f)
            for (int lv = 0; lv <= kMaxDepth; ++lv) {
                double h = 2.0 * P.fmm[f].R / (double)(1 << lv);
                itilde_all(P.p, P.fmm[f].lam_s * P.fmm[f].lam_s * h * h, buf);
                for (int n = 0; n <= P.p; ++n) is[f * per + lv * (LPB_MAX_P + 1) + n] = 1.0 / buf[n];
                itilde_all(P.p, P.fmm[f].lam_t * P.fmm[f].lam_t * h * h, buf);
                for (int n = 0; n <= P.p; ++n) it[f * per + lv * (LPB_MAX_P + 1) + n] = 1.0 / buf[n];
            }
        UP(bes_tab, tb);
        UP(ith_s, is);
        UP(ith_t, it);
        // 4 pi i_n(lam h) of every FMM and level (the W- and X-list kernels)
        std::vector<double> fs(P.fmm.size() * per, 0.0), ft(P.fmm.size() * per, 0.0);
        for (size_t f = 0; f < P.fmm.size(); ++f)
            for (int lv = 0; lv <= kMaxDepth; ++lv) {
                double h = 2.0 * P.fmm[f].R / (double)(1 << lv);
                bessel_i_all(P.p, P.fmm[f].lam_s * h, buf);
                for (int n = 0; n <= P.p; ++n) fs[f * per + lv * (LPB_MAX_P + 1) + n] = 4.0 * LPB_PI * buf[n];
                bessel_i_all(P.p, P.fmm[f].lam_t * h, buf);
                for (int n = 0; n <= P.p; ++n) ft[f * per + lv * (LPB_MAX_P + 1) + n] = 4.0 * LPB_PI * buf[n];
            }
        UP(fin_s, fs);
        UP(fin_t, ft);
    }
    A.n_tiles = (int)P.tiles.size();
    // work lists
    std::vector<int> p2m, l2p, pfree, rleaf, rslot, m2lb;
    for (size_t i = 0; i < P.sl_me.size(); ++i)
        if (P.sl_me[i] >= 0) p2m.push_back((int)i);
    // free-space near field: a work item is T <= 64 targets of one leaf on T x S
    // lanes of a 64-lane block, each target's sources split S ways.  A leaf of
    // n targets takes P >= ceil(n / 64) items of T = ceil(n / P) targets,
    // S = min(4, 64 / T), with P minimising the lane-passes over the sources
    // P / S (ties: fewer items), so that few lanes idle (a leaf of 40 takes 2
    // items of 20 x 3 instead of 2 passes of 32 lanes); most source-heavy
    // items first.  (S saturates at T <= 16, so P beyond ceil(n / 16) never
    // helps.)
    std::vector<int> pfree_t0, pfree_ts;
    {
        std::vector<std::array<int64_t, 4>> wl;   // (-cost class, leaf, first target, T | S << 8)
        for (size_t i = 0; i < P.tl_le.size(); ++i) {
            if (P.p2p_ptr[i + 1] == P.p2p_ptr[i]) continue;
            int64_t ns = 0;
            for (int k = P.p2p_ptr[i]; k < P.p2p_ptr[i + 1]; ++k) ns += P.sl_start[P.p2p_src[k] + 1] - P.sl_start[P.p2p_src[k]];
            const int n = P.tl_start[i + 1] - P.tl_start[i];
            int bestP = 1, bestS = 1;
            double best = 1e30;
            const int np0 = std::max(1, (n + 63) / 64), np1 = std::min(n, (n + 15) / 16 + 1);
            bestP = np0;
            for (int np = np0; np <= np1; ++np) {
                const int nt = (n + np - 1) / np;
                if (nt > 64) continue;
                const int S = std::max(1, std::min(4, 64 / nt));
                const double cost = (double)np / S;
                if (cost < best - 1e-12) {
                    best = cost;
                    bestP = np;
                    bestS = S;
                }
            }
            const int nt = (n + bestP - 1) / bestP;
            for (int t = P.tl_start[i]; t < P.tl_start[i + 1]; t += nt) {
                // cost class: floor(log2(lane passes)); within a class the leaf order (locality) is kept
                int64_t passes = (ns + bestS - 1) / bestS, cls = 0;
                while ((passes >> (cls + 1)) > 0) ++cls;
                wl.push_back({-cls, (int64_t)i, (int64_t)t, (int64_t)(nt | (bestS << 8))});
            }
        }
        std::stable_sort(wl.begin(), wl.end(), [](const std::array<int64_t, 4>& a, const std::array<int64_t, 4>& b) {
            return a[0] < b[0];
        });
        for (auto& w : wl) {
            pfree.push_back((int)w[1]);
            pfree_t0.push_back((int)w[2]);
            pfree_ts.push_back((int)w[3]);
        }
    }
    for (size_t i = 0; i < P.tl_le.size(); ++i) {
        if (P.tl_le[i] >= 0) l2p.push_back((int)i);
        if (P.rp_ptr[i + 1] > P.rp_ptr[i])
            for (int j = P.tl_start[i]; j < P.tl_start[i + 1]; ++j) {
                rleaf.push_back((int)i);
                rslot.push_back(j);
            }
    }
    for (int i = 0; i < P.n_le; ++i)
        if (P.m2l_ptr[i + 1] > P.m2l_ptr[i]) m2lb.push_back(i);
    UP(p2m_leaves, p2m);
    UP(l2p_leaves, l2p);
    UP(p2p_free_leaves, pfree);
    UP(p2p_free_t0, pfree_t0);
    UP(p2p_free_ts, pfree_ts);
    UP(react_tgt_leaf, rleaf);
    UP(react_tgt_slot, rslot);
    UP(m2l_boxes, m2lb);
#undef UP
    A.n_react_targets = (int)rleaf.size();
    c->sched.n_p2m = (int)p2m.size();
    c->sched.n_l2p = (int)l2p.size();
    // leaves per 64-lane block of the fixed-order P2M / L2P: 64 / nl lanes per
    // leaf, the choice with fewer lane-passes over the leaves' points
    auto pick_nl = [](const std::vector<int>& leaves, const std::vector<int>& start) {
        int64_t c2 = 0, c4 = 0;
        for (int i : leaves) {
            const int64_t n = start[i + 1] - start[i];
            c2 += (n + 31) / 32 * 32;
            c4 += (n + 15) / 16 * 16;
        }
        return c4 < c2 ? 4 : 2;
    };
    c->sched.p2m_nl = pick_nl(p2m, P.sl_start);
    c->sched.l2p_nl = pick_nl(l2p, P.tl_start);
    c->sched.n_p2p_free = (int)pfree.size();
    c->sched.n_m2l_boxes = (int)m2lb.size();
    for (int l = 0; l <= kMaxDepth + 1; ++l) {
        c->sched.bm2m_lv[l] = P.bm2m_lv[l];
        c->sched.bl2l_lv[l] = P.bl2l_lv[l];
    }
    c->sched.bm2l_w0 = P.bm2l_w0;
    c->sched.bm2l_w1 = P.bm2l_w1;
    // the points, from the builder's sets
    {
        int *scidx, *tcidx, *tout;
        T* su[6] = {};
        T* tu[6] = {};
        const size_t ns = (size_t)P.n_spts, nt = (size_t)P.n_tpts;
        if ((s = dalloc<int>(c, c->plan_bufs, ns, &scidx)) != LPB_OK) return s;
        if ((s = dalloc<int>(c, c->plan_bufs, nt, &tcidx)) != LPB_OK) return s;
        if ((s = dalloc<int>(c, c->plan_bufs, nt, &tout)) != LPB_OK) return s;
        for (int d = 0; d < (sizeof(T) == 4 ? 6 : 3); ++d) {
            if ((s = dalloc<T>(c, c->plan_bufs, ns, &su[d])) != LPB_OK) return s;
            if ((s = dalloc<T>(c, c->plan_bufs, nt, &tu[d])) != LPB_OK) return s;
        }
        std::string msg;
        if (!pb.gather<T>(P.s_sets, nullptr, P.ncharges, P.n_spts, scidx, nullptr, su[0], su[1], su[2], su[3], su[4], su[5],
                          msg) ||
            !pb.gather<T>(P.t_sets, &P.t_set_slot, P.ncharges, P.n_tpts, tcidx, tout, tu[0], tu[1], tu[2], tu[3], tu[4],
                          tu[5], msg))
            return fail(c, (lpb_status)pb.failure(), msg);
        A.s_cidx = scidx;
        A.t_cidx = tcidx;
        A.t_out = tout;
        A.s_ux = su[0]; A.s_uy = su[1]; A.s_uz = su[2]; A.s_lx = su[3]; A.s_ly = su[4]; A.s_lz = su[5];
        A.t_ux = tu[0]; A.t_uy = tu[1]; A.t_uz = tu[2]; A.t_lx = tu[3]; A.t_ly = tu[4]; A.t_lz = tu[5];
    }
    T* qs;
    if ((s = dalloc<T>(c, c->plan_bufs, (size_t)P.n_spts, &qs)) != LPB_OK) return s;
    A.qs = qs;
    T *me, *le;
    // one extra zero row after the last box of each (missing sources of the batched products read it)
    if ((s = dalloc<T>(c, c->plan_bufs, (size_t)(P.n_me + 1) * A.KP, &me)) != LPB_OK) return s;
    if ((s = dalloc<T>(c, c->plan_bufs, (size_t)(P.n_le + 1) * A.KP, &le)) != LPB_OK) return s;
    HIPCHK(c, hipMemset(le, 0, sizeof(T) * (size_t)(P.n_le + 1) * A.KP));
    // the padding rows k >= K of the expansions are read by the tiled M2L and must stay zero
    HIPCHK(c, hipMemset(me, 0, sizeof(T) * (size_t)(P.n_me + 1) * A.KP));
    A.me = me;
    A.le = le;
    A.n_le = P.n_le;
    A.n_me = P.n_me;
    T* scr = nullptr;
    if (!P.m2l_src.empty())
        if ((s = dalloc<T>(c, c->plan_bufs, P.m2l_src.size() * (size_t)A.K, &scr)) != LPB_OK) return s;
    A.m2l_scratch = scr;
    double* parts;
    if ((s = dalloc<double>(c, c->plan_bufs, (size_t)(P.nslots + 1) * P.ncharges, &parts)) != LPB_OK) return s;
    A.parts = parts;
    if ((s = dalloc<double>(c, c->plan_bufs, (size_t)P.ncharges, &c->d_q)) != LPB_OK) return s;
    if ((s = dalloc<double>(c, c->plan_bufs, (size_t)P.ncharges, &c->d_phi)) != LPB_OK) return s;
    A.q = c->d_q;
    A.phi = c->d_phi;
    A.gl_x = (const double*)c->d_glx.ptr;
    A.gl_w = (const double*)c->d_glw.ptr;
    return LPB_OK;
}

lpb_status build_and_upload(lpb_ctx* c)
{
    auto t0 = std::chrono::steady_clock::now();
    drop_graph(c);
    c->tune_needed = true;
    c->prepared = false;
    free_bufs(c, c->plan_bufs);
    free_bufs(c, c->op_bufs);
    c->ops_dirty = true;
    c->have_tree = false;
    Plan& P = c->plan;
    P.p = c->opt.p;
    P.K = (P.p + 1) * (P.p + 1);
    P.leaf_cap = c->opt.leaf_cap;
    P.adaptive = c->opt.adaptive;
    int st = 0;
    // the points go through the device builder (its buffers are the
    // context's, returned when it goes out of scope)
    DevPointBuilder pb(c->stream, [c](size_t b) { return dev_alloc(c, b); }, [c](void* p) { dev_free(c, p); });
    std::string msg;
    if (!pb.set_coords(c->xs, c->ys, c->zs, msg)) return fail(c, (lpb_status)pb.failure(), msg);
    msg = build_plan(P, c->media, c->xs, c->ys, c->zs, c->opt.iface_tol, pb, &st);
    if (st != LPB_OK) return fail(c, (lpb_status)st, msg);
    lpb_status s = (c->opt.precision == LPB_MIXED) ? fill_args<float>(c, c->a32, pb) : fill_args<double>(c, c->a64, pb);
    if (s != LPB_OK) {
        free_bufs(c, c->plan_bufs);
        return s;
    }
    c->have_tree = true;
    c->stats.n_fmm = (int)P.fmm.size();
    c->stats.max_depth = P.max_depth;
    c->stats.n_m2l_pairs = P.n_m2l_pairs;
    c->stats.n_m2l_tile_pairs = P.n_m2l_tile_pairs;
    c->stats.n_m2l_tiles = (int64_t)P.tiles.size();
    c->stats.n_p2p_pairs = P.n_p2p_pairs;
    c->stats.n_react_p2p_pairs = P.n_react_p2p_pairs;
    c->stats.n_operators = (int64_t)P.ops.size();
    {
        // links of the batched M2M / L2L items (valid source rows) and the
        // distinct operators of the untiled V-list pairs
        auto links = [&](int w0, int w1) {
            int64_t k = 0;
            for (int w = w0; w < w1; ++w)
                for (int t = P.bw_term_ptr[w]; t < P.bw_term_ptr[w + 1]; ++t)
                    for (int j = 0; j < 64; ++j) k += (P.bw_src[64 * (size_t)t + j] >= 0 && P.bw_dst[64 * (size_t)w + j] >= 0);
            return k;
        };
        c->stats.n_m2m_links = links(P.bm2m_lv[0], P.bm2m_lv[kMaxDepth + 1]);
        c->stats.n_l2l_links = links(P.bl2l_lv[0], P.bl2l_lv[kMaxDepth + 1]);
        std::vector<int> ops(P.m2l_op);
        std::sort(ops.begin(), ops.end());
        c->stats.n_m2l_list_ops = (int64_t)(std::unique(ops.begin(), ops.end()) - ops.begin());
        c->stats.n_p2m_points = P.n_spts;
        c->stats.n_l2p_points = P.n_tpts;
        c->stats.n_w_pairs = P.n_w_pairs;
        c->stats.n_x_pairs = P.n_x_pairs;
        c->stats.n_w_points = P.n_w_points;
        c->stats.n_x_points = P.n_x_points;
        c->stats.n_point_ops = (int64_t)P.pt_ops.size();
    }
    c->stats.t_build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return LPB_OK;
}

lpb_status generate_operators_impl(lpb_ctx* c);

// Operators of the current plan; on failure no operator buffer is kept.
lpb_status generate_operators(lpb_ctx* c)
{
    lpb_status s = generate_operators_impl(c);
    if (s != LPB_OK) free_bufs(c, c->op_bufs);
    return s;
}

lpb_status generate_operators_impl(lpb_ctx* c)
{
    Plan& P = c->plan;
    drop_graph(c);
    c->tune_needed = true;
    c->prepared = false;
    free_bufs(c, c->op_bufs);
    const int K = P.K, Kp = (P.p + 1) * (P.p + 2) / 2;
    lpb_status s;
    std::vector<int> freel, reactl, rfl, rfidx(P.fmm.size(), -1);
    for (size_t i = 0; i < P.ops.size(); ++i) (P.ops[i].type == OP_M2L_REACT ? reactl : freel).push_back((int)i);
    for (size_t i = 0; i < P.fmm.size(); ++i)
        if (P.fmm[i].kind == 1) {
            rfidx[i] = (int)rfl.size();
            rfl.push_back((int)i);
        }
    OpgenInputs& g = c->og;
    g = OpgenInputs{};
    g.p = P.p;
    g.n_ops = (int)P.ops.size();
    g.n_rkeys = (int)P.rkeys.size();
    g.n_rf = (int)rfl.size();
    g.n_free = (int)freel.size();
    g.n_react = (int)reactl.size();
    g.quad_tol = c->opt.quad_tol;
    OpDesc* dops;
    RKey* drk;
    int *dfl, *drl, *drf, *drfi;
    if ((s = upload(c, c->op_bufs, P.ops, &dops)) != LPB_OK) return s;
    if ((s = upload(c, c->op_bufs, P.rkeys, &drk)) != LPB_OK) return s;
    if ((s = upload(c, c->op_bufs, freel, &dfl)) != LPB_OK) return s;
    if ((s = upload(c, c->op_bufs, reactl, &drl)) != LPB_OK) return s;
    if ((s = upload(c, c->op_bufs, rfl, &drf)) != LPB_OK) return s;
    if ((s = upload(c, c->op_bufs, rfidx, &drfi)) != LPB_OK) return s;
    g.d_ops = dops; g.d_rkeys = drk; g.d_free_list = dfl; g.d_react_list = drl; g.d_rf_list = drf; g.d_rf_index = drfi;
    g.d_fmm = (c->opt.precision == LPB_MIXED) ? c->a32.fmm : c->a64.fmm;
    g.d_media = (c->opt.precision == LPB_MIXED) ? c->a32.media : c->a64.media;
    g.d_btab = (const double*)c->d_btab.ptr;
    g.d_gtab = (const double*)c->d_gtab.ptr;
    const int N1 = 2 * P.p + 4;
    if ((s = dalloc<double>(c, c->op_bufs, (size_t)g.n_rf * Kp * K * (P.p + 2), &g.d_dtab)) != LPB_OK) return s;
    if ((s = dalloc<double>(c, c->op_bufs, (size_t)g.n_rkeys * 4 * N1 * N1, &g.d_stab)) != LPB_OK) return s;
    if ((s = dalloc<double>(c, c->op_bufs, (size_t)g.n_ops * K * K, &g.d_pool)) != LPB_OK) return s;
    if (g.n_rkeys > 0) HIPCHK(c, hipMemsetAsync(g.d_stab, 0, sizeof(double) * (size_t)g.n_rkeys * 4 * N1 * N1, c->stream));
    g.d_pool32 = nullptr;
    g.d_flag = (int*)c->d_flag.ptr;
    g.KP = (K + 15) / 16 * 16;
    g.n_swz = (int)P.swz_ops.size();
    int* dswz;
    if ((s = upload(c, c->op_bufs, P.swz_ops, &dswz)) != LPB_OK) return s;
    g.d_swz_ops = dswz;
    g.d_swz64 = nullptr;
    g.d_swz32 = nullptr;
    g.n_orb = 0;
    g.NRB = class_row_blocks(P.p);
    g.d_orb_ops = nullptr;
    g.d_rowmap = nullptr;
    g.d_orb32 = nullptr;
    if (c->opt.precision == LPB_MIXED) {
        if ((s = dalloc<float>(c, c->op_bufs, (size_t)g.n_swz * g.KP * g.KP, &g.d_swz32)) != LPB_OK) return s;
        if (P.p >= kOrbitMinP && P.p <= kOrbitMaxP && !P.orb_ops.empty()) {
            int *dob, *drm;
            g.n_orb = (int)P.orb_ops.size();
            if ((s = upload(c, c->op_bufs, P.orb_ops, &dob)) != LPB_OK) return s;
            if ((s = upload(c, c->op_bufs, class_rowmap(P.p), &drm)) != LPB_OK) return s;
            g.d_orb_ops = dob;
            g.d_rowmap = drm;
            if ((s = dalloc<float>(c, c->op_bufs, (size_t)g.n_orb * g.NRB * 16 * g.KP, &g.d_orb32)) != LPB_OK) return s;
        }
    } else {
        if ((s = dalloc<double>(c, c->op_bufs, (size_t)g.n_swz * g.KP * g.KP, &g.d_swz64)) != LPB_OK) return s;
    }
    // reaction point operators of adaptive trees (kept for the evaluations)
    g.n_pt = (int)P.pt_ops.size();
    g.d_pt_ops = nullptr;
    g.d_pt_vec = nullptr;
    g.pt_f32 = c->opt.precision == LPB_MIXED;
    if (g.n_pt > 0) {
        PointOp* dpo;
        if ((s = upload(c, c->op_bufs, P.pt_ops, &dpo)) != LPB_OK) return s;
        g.d_pt_ops = dpo;
        if ((s = dalloc<double>(c, c->op_bufs, (size_t)g.n_pt * K, &g.d_pt_vec)) != LPB_OK) return s;
        auto coords = [&](const auto& A) {
            const void* t[6] = {A.t_ux, A.t_uy, A.t_uz, A.t_lx, A.t_ly, A.t_lz};
            const void* u[6] = {A.s_ux, A.s_uy, A.s_uz, A.s_lx, A.s_ly, A.s_lz};
            for (int d = 0; d < 6; ++d) {
                g.t_u[d] = t[d];
                g.s_u[d] = u[d];
            }
            g.tl_ctr = A.tl_ctr;
            g.sl_ctr = A.sl_ctr;
        };
        if (c->opt.precision == LPB_MIXED) coords(c->a32);
        else coords(c->a64);
    }
    HIPCHK(c, hipMemsetAsync(g.d_flag, 0, sizeof(int), c->stream));
    HIPCHK(c, hipEventRecord(c->ev0, c->stream));
    HIPCHK(c, opgen_run(g, c->stream));
    HIPCHK(c, hipEventRecord(c->ev1, c->stream));
    int flag = 0;
    HIPCHK(c, hipMemcpyAsync(&flag, g.d_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
    c->stats.t_opgen_ms = ms;
    if (flag & 1) return fail(c, LPB_ENUMERIC, "Sommerfeld quadrature panel budget exceeded");
    if (flag & 2) return fail(c, LPB_ENUMERIC, "forward recurrence stability bound violated");
    // the kernels read the operators in the MFMA operand layout only; the
    // FP64 master copy is no longer needed
    for (auto& b : c->op_bufs)
        if (b.ptr == (void*)g.d_pool) free_buf(c, b);
    c->a32.pt_vec = g.d_pt_vec;
    c->a64.pt_vec = g.d_pt_vec;
    if (c->opt.precision == LPB_MIXED) {
        c->a32.pool_swz = g.d_swz32;
        c->a32.pool_orb = g.d_orb32;
        c->stats.operator_bytes = ((int64_t)g.n_swz * g.KP * g.KP + (int64_t)g.n_orb * g.NRB * 16 * g.KP) *
                                  (int64_t)sizeof(float);
    } else {
        c->a64.pool_swz = g.d_swz64;
        c->stats.operator_bytes = (int64_t)g.n_swz * g.KP * g.KP * (int64_t)sizeof(double);
    }
    c->ops_dirty = false;
    return LPB_OK;
}

// Schedule autotuning: time each block -> work schedule of the two
// matrix-core stages (3 launches each, best of 3) and keep the fastest.
// The candidates permute which block computes which work item, or (tiled
// M2L) split the same products over more waves; results do not change.
template <typename T>
lpb_status autotune(lpb_ctx* c, EvalArgs<T>& A)
{
    auto t0 = std::chrono::steady_clock::now();
    int* field[2] = {&A.tile_sched, &A.batch_sched};
    // tiled M2L candidates: order bit 0 with, where the orbit form exists
    // (mixed precision, kOrbitMinP <= p <= kOrbitMaxP), the orbit form with
    // operands in LDS or in registers (bit 3) -- these give the
    // same bits -- and, with autotune = 2, also the per-offset form (bit 2)
    // with one or four waves per row block (bit 1), whose sums round
    // differently; elsewhere the per-offset form's bits 0-1.  Batched
    // translations: order bit 0, resident-block grid bits 1-2.
    std::vector<int> tile_cands;
    const bool orbit = sizeof(T) == 4 && A.pool_orb && A.p >= kOrbitMinP && A.p <= kOrbitMaxP;
    if (orbit) {
        tile_cands = {0, 1, 8, 9};
        if (c->opt.autotune == 2) tile_cands.insert(tile_cands.end(), {4, 5, 6, 7});
    } else {
        tile_cands = {0, 1, 2, 3};
    }
    for (int which = 0; which < 2; ++which) {
        float best = 1e30f;
        int pick = 0;
        const int ncand = which == 0 ? (int)tile_cands.size() : 8;
        for (int ci = 0; ci < ncand; ++ci) {
            const int sc = which == 0 ? tile_cands[ci] : ci;
            *field[which] = sc;
            float tmin = 1e30f;
            for (int rep = 0; rep < 3; ++rep) {
                HIPCHK(c, hipEventRecord(c->ev0, c->stream));
                hipError_t e = stage_run<T>(A, c->sched, which, c->stream);
                if (e != hipSuccess) return fail(c, LPB_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
                HIPCHK(c, hipEventRecord(c->ev1, c->stream));
                HIPCHK(c, hipEventSynchronize(c->ev1));
                float ms = 0.f;
                HIPCHK(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
                tmin = std::min(tmin, ms);
            }
            if (tmin < best) {
                best = tmin;
                pick = sc;
            }
        }
        *field[which] = pick;
    }
    c->stats.tile_schedule = A.tile_sched;
    c->stats.batch_schedule = A.batch_sched;
    c->stats.t_tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return LPB_OK;
}

template <typename T>
lpb_status run_eval_t(lpb_ctx* c, EvalArgs<T>& A)
{
    if (c->tune_needed) {
        if (c->opt.autotune) {
            lpb_status s = autotune<T>(c, A);
            if (s != LPB_OK) return s;
        } else {
            A.tile_sched = c->opt.schedule & 15;
            A.batch_sched = (c->opt.schedule >> 4) & 15;
            c->stats.tile_schedule = A.tile_sched;
            c->stats.batch_schedule = A.batch_sched;
        }
        c->tune_needed = false;
        drop_graph(c);
    }
    const bool use_graph = c->opt.graph && !c->opt.timing;
    if (use_graph && !c->gexec) {
        // every pass is a kernel (no memset nodes); the schedules and buffers
        // it captures stay fixed until the next tree or operator change
        HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = eval_run<T>(A, c->sched, c->opt.stages, c->stream, nullptr, &c->fork);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(c->stream, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return fail(c, LPB_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
        }
        c->graph = g;
        HIPCHK(c, hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0));
    }
    HIPCHK(c, hipEventRecord(c->ev0, c->stream));
    if (use_graph) {
        HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
    } else {
        hipEvent_t* ev = c->opt.timing ? c->evs : nullptr;
        hipError_t e = eval_run<T>(A, c->sched, c->opt.stages, c->stream, ev, &c->fork);
        if (e != hipSuccess) return fail(c, LPB_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    }
    HIPCHK(c, hipEventRecord(c->ev1, c->stream));
    return LPB_OK;
}

lpb_status run_eval(lpb_ctx* c)
{
    return (c->opt.precision == LPB_MIXED) ? run_eval_t<float>(c, c->a32) : run_eval_t<double>(c, c->a64);
}

// The evaluation passes of a prepared context launched one by one, with the
// partial potentials in `parts` (the GPU's scratch array), charges read from
// q and the sum written to phi (caller device memory).
template <typename T>
lpb_status run_noalloc_t(lpb_ctx* c, const EvalArgs<T>& A0, const double* q, double* phi, double* parts)
{
    EvalArgs<T> A = A0;
    A.q = q;
    A.phi = phi;
    A.parts = parts;
    HIPCHK(c, hipEventRecord(c->ev0, c->stream));
    hipError_t e = eval_run<T>(A, c->sched, c->opt.stages, c->stream, nullptr, &c->fork);
    if (e != hipSuccess) return fail(c, LPB_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    HIPCHK(c, hipEventRecord(c->ev1, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
    c->stats.t_eval_ms = ms;
    return LPB_OK;
}

}  // namespace

extern "C" {

void lpb_default_options(lpb_options* opt)
{
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->p = 10;
    opt->leaf_cap = 50;
    opt->precision = LPB_FP64;
    opt->quad_tol = 1e-16;
    opt->iface_tol = 1e-9;
    opt->device = 0;
    opt->stream = nullptr;
    opt->stages = 3;
    opt->timing = 0;
    opt->graph = 1;
    opt->autotune = 1;
}

lpb_status lpb_create(const lpb_options* opt, lpb_ctx** out)
{
    if (!out) return fail(nullptr, LPB_EINVAL, "out is NULL");
    *out = nullptr;
    lpb_options o;
    lpb_default_options(&o);
    if (opt) o = *opt;
    if (o.precision != LPB_FP64 && o.precision != LPB_MIXED) return fail(nullptr, LPB_EINVAL, "bad precision");
    if (o.p < 1 || o.p > LPB_MAX_P) return fail(nullptr, LPB_ERANGE, "p out of range");
    if (o.precision == LPB_FP64 && o.p > LPB_MAX_P_FP64)
        return fail(nullptr, LPB_ERANGE, "p above LPB_MAX_P_FP64 in FP64 (the FP64 operand slab of a block would exceed LDS)");
    if (o.leaf_cap < 1) return fail(nullptr, LPB_ERANGE, "leaf_cap must be >= 1");
    if (!(o.quad_tol > 0.0 && o.quad_tol < 1e-3)) return fail(nullptr, LPB_EINVAL, "quad_tol out of range");
    if (!(o.iface_tol >= 0.0)) return fail(nullptr, LPB_EINVAL, "iface_tol must be >= 0");
    if (!o.alloc != !o.free) return fail(nullptr, LPB_EINVAL, "alloc and free must be set together");
    if (o.autotune < 0 || o.autotune > 2) return fail(nullptr, LPB_EINVAL, "autotune must be 0, 1 or 2");
    if (o.schedule < 0 || (o.schedule >> 4) > 7)
        return fail(nullptr, LPB_EINVAL, "schedule codes out of range");
    if (o.adaptive < 0 || o.adaptive > 2) return fail(nullptr, LPB_EINVAL, "adaptive must be 0, 1 or 2");
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= 0) return fail(nullptr, LPB_EDEVICE, "no HIP device available");
    if (o.device < 0 || o.device >= ndev) return fail(nullptr, LPB_EINVAL, "device ordinal out of range");
    // on failure below, everything the context holds so far is released
    struct Releaser {
        lpb_ctx* c;
        ~Releaser() { if (c) lpb_destroy(c); }
    } guard{new lpb_ctx()};
    lpb_ctx* c = guard.c;
    c->opt = o;
    c->stream = (hipStream_t)o.stream;
    e = hipSetDevice(o.device);
    if (e != hipSuccess) return fail(nullptr, LPB_EDEVICE, hipGetErrorString(e));
    e = scratch_init(o.device);
    if (e != hipSuccess) return fail(nullptr, LPB_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    if (o.graph && !c->stream) {
        // graphs cannot be captured on the null stream: use a blocking stream of
        // our own (it orders itself with the null stream)
        if (hipStreamCreate(&c->own_stream) != hipSuccess) return fail(nullptr, LPB_EDEVICE, "stream create failed");
        c->stream = c->own_stream;
    }
    if (opgen_upload_constants() != hipSuccess) return fail(nullptr, LPB_EDEVICE, "constant upload failed");
    make_btab(o.p, c->btab);
    make_gtab(o.p, c->gtab);
    auto up = [&](const std::vector<double>& v, DevBuf& b) -> lpb_status {
        b.bytes = v.size() * sizeof(double);
        b.ptr = dev_alloc(c, std::max<size_t>(b.bytes, 8));
        if (!b.ptr) return LPB_ENOMEM;
        return hipMemcpy(b.ptr, v.data(), b.bytes, hipMemcpyHostToDevice) == hipSuccess ? LPB_OK : LPB_EDEVICE;
    };
    double glx[20], glw[20];
    gauss_legendre20(glx, glw);
    for (auto t : {std::make_pair(&c->btab, &c->d_btab), std::make_pair(&c->gtab, &c->d_gtab)}) {
        lpb_status s = up(*t.first, *t.second);
        if (s != LPB_OK) return fail(nullptr, s, "table upload failed");
    }
    {
        lpb_status s = up(std::vector<double>(glx, glx + 20), c->d_glx);
        if (s == LPB_OK) s = up(std::vector<double>(glw, glw + 20), c->d_glw);
        if (s != LPB_OK) return fail(nullptr, s, "table upload failed");
    }
    c->d_flag.ptr = dev_alloc(c, 256);
    if (!c->d_flag.ptr) return fail(nullptr, LPB_ENOMEM, "flag alloc failed");
    if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess)
        return fail(nullptr, LPB_EDEVICE, "event create failed");
    for (auto& e : c->evs)
        if (hipEventCreate(&e) != hipSuccess) return fail(nullptr, LPB_EDEVICE, "event create failed");
    if (hipStreamCreateWithFlags(&c->fork.side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->fork.fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->fork.join, hipEventDisableTiming) != hipSuccess ||
        hipStreamCreateWithFlags(&c->fork.near, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->fork.near_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->fork.near_join, hipEventDisableTiming) != hipSuccess)
        return fail(nullptr, LPB_EDEVICE, "side stream create failed");
    *out = c;
    guard.c = nullptr;
    return LPB_OK;
}

lpb_status lpb_set_layers(lpb_ctx* c, int n_layers, const double* eps, const double* lambda, const double* interfaces)
{
    if (!c) return LPB_EINVAL;
    if (c->batched) return fail(c, LPB_ESTATE, "context is batched; use lpb_set_systems");
    Medium M;
    lpb_status s = check_layers(c, n_layers, eps, lambda, interfaces, M);
    if (s != LPB_OK) return s;
    HIPCHK(c, hipSetDevice(c->opt.device));
    c->media.assign(1, M);
    c->have_layers = true;
    c->ops_dirty = true;
    c->prepared = false;
    if (c->xs.size() == 1) return build_and_upload(c);
    return LPB_OK;
}

lpb_status lpb_build_tree(lpb_ctx* c, int64_t n, const double* x, const double* y, const double* z, int on_device)
{
    if (!c) return LPB_EINVAL;
    if (c->batched) return fail(c, LPB_ESTATE, "context is batched; use lpb_build_trees");
    if (!c->have_layers) return fail(c, LPB_ESTATE, "lpb_set_layers must come first");
    HIPCHK(c, hipSetDevice(c->opt.device));
    std::vector<double> X, Y, Z;
    lpb_status s = read_coords(c, n, x, y, z, on_device, X, Y, Z);
    if (s != LPB_OK) return s;
    c->xs.assign(1, std::move(X));
    c->ys.assign(1, std::move(Y));
    c->zs.assign(1, std::move(Z));
    s = build_and_upload(c);
    if (s != LPB_OK) {
        c->xs.clear(); c->ys.clear(); c->zs.clear();
    }
    return s;
}

static lpb_status evaluate_common(lpb_ctx* c, int nsys, const double* const* q, double* const* phi, int on_device)
{
    HIPCHK(c, hipSetDevice(c->opt.device));
    Plan& P = c->plan;
    for (int s = 0; s < nsys; ++s) {
        int64_t n = P.sys_charge_off[s + 1] - P.sys_charge_off[s];
        if (n > 0 && (!q[s] || !phi[s])) return fail(c, LPB_EINVAL, "null q or phi");
    }
    if (c->ops_dirty) {
        lpb_status st = generate_operators(c);
        if (st != LPB_OK) return st;
    }
    for (int s = 0; s < nsys; ++s) {
        int64_t n = P.sys_charge_off[s + 1] - P.sys_charge_off[s];
        if (n == 0) continue;
        HIPCHK(c, hipMemcpyAsync(c->d_q + P.sys_charge_off[s], q[s], n * sizeof(double),
                                 on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
    }
    lpb_status st = run_eval(c);
    if (st != LPB_OK) return st;
    for (int s = 0; s < nsys; ++s) {
        int64_t n = P.sys_charge_off[s + 1] - P.sys_charge_off[s];
        if (n == 0) continue;
        HIPCHK(c, hipMemcpyAsync(phi[s], c->d_phi + P.sys_charge_off[s], n * sizeof(double),
                                 on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->prepared = true;
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
    c->stats.t_eval_ms = ms;
    if (c->opt.timing)
        for (int k = 0; k < 10; ++k) {
            float t = 0.f;
            HIPCHK(c, hipEventElapsedTime(&t, c->evs[k], c->evs[k + 1]));
            c->stats.t_stage_ms[k] = t;
        }
    return LPB_OK;
}

lpb_status lpb_evaluate(lpb_ctx* c, const double* q, double* phi, int on_device)
{
    if (!c) return LPB_EINVAL;
    if (c->batched) return fail(c, LPB_ESTATE, "context is batched; use lpb_evaluate_batch");
    if (!c->have_layers || !c->have_tree) return fail(c, LPB_ESTATE, "set_layers and build_tree must come first");
    if (q && phi && (const void*)q == (const void*)phi) return fail(c, LPB_EINVAL, "phi aliases q");
    return evaluate_common(c, 1, &q, &phi, on_device);
}

lpb_status lpb_evaluate_noalloc(lpb_ctx* c, const double* q, double* phi)
{
    if (!c) return LPB_EINVAL;
    if (c->batched) return fail(c, LPB_ESTATE, "lpb_evaluate_noalloc takes single-system contexts");
    if (!c->have_layers || !c->have_tree || c->ops_dirty || !c->prepared)
        return fail(c, LPB_ESTATE, "context not prepared: run lpb_evaluate once after lpb_set_layers / lpb_build_tree");
    const Plan& P = c->plan;
    const uint64_t need = (uint64_t)(P.nslots + 1) * (uint64_t)P.ncharges;
    if (need > (uint64_t)LPB_NOALLOC_MAX_PARTS)
        return fail(c, LPB_ERANGE, "n_slots * n = " + std::to_string(need) + " partial potentials exceed LPB_NOALLOC_MAX_PARTS = " +
                                       std::to_string((uint64_t)LPB_NOALLOC_MAX_PARTS));
    if (P.ncharges == 0) return LPB_OK;
    if (!q || !phi) return fail(c, LPB_EINVAL, "null q or phi");
    if ((const void*)q == (const void*)phi) return fail(c, LPB_EINVAL, "phi aliases q");
    double* parts = scratch_ptr(c->opt.device);
    if (!parts) return fail(c, LPB_ESTATE, "scratch array of this device not initialised");
    HIPCHK(c, hipSetDevice(c->opt.device));
    return (c->opt.precision == LPB_MIXED) ? run_noalloc_t<float>(c, c->a32, q, phi, parts)
                                           : run_noalloc_t<double>(c, c->a64, q, phi, parts);
}

lpb_status lpb_set_systems(lpb_ctx* c, int n_sys, const int* n_layers, const double* const* eps,
                           const double* const* lambda, const double* const* interfaces)
{
    if (!c) return LPB_EINVAL;
    if (n_sys < 1 || !n_layers || !eps || !lambda || !interfaces) return fail(c, LPB_EINVAL, "bad system arrays");
    std::vector<Medium> ms(n_sys);
    for (int s = 0; s < n_sys; ++s) {
        lpb_status st = check_layers(c, n_layers[s], eps[s], lambda[s], interfaces[s], ms[s]);
        if (st != LPB_OK) return st;
    }
    HIPCHK(c, hipSetDevice(c->opt.device));
    c->batched = true;
    c->media = ms;
    c->have_layers = true;
    c->ops_dirty = true;
    if ((int)c->xs.size() == n_sys) return build_and_upload(c);
    c->xs.clear(); c->ys.clear(); c->zs.clear();
    c->have_tree = false;
    return LPB_OK;
}

lpb_status lpb_build_trees(lpb_ctx* c, int n_sys, const int64_t* n, const double* const* x, const double* const* y,
                           const double* const* z, int on_device)
{
    if (!c) return LPB_EINVAL;
    if (!c->batched || !c->have_layers) return fail(c, LPB_ESTATE, "lpb_set_systems must come first");
    if (n_sys != (int)c->media.size() || !n || !x || !y || !z) return fail(c, LPB_EINVAL, "bad system arrays");
    HIPCHK(c, hipSetDevice(c->opt.device));
    std::vector<std::vector<double>> X(n_sys), Y(n_sys), Z(n_sys);
    for (int s = 0; s < n_sys; ++s) {
        lpb_status st = read_coords(c, n[s], x[s], y[s], z[s], on_device, X[s], Y[s], Z[s]);
        if (st != LPB_OK) return st;
    }
    c->xs = std::move(X);
    c->ys = std::move(Y);
    c->zs = std::move(Z);
    lpb_status st = build_and_upload(c);
    if (st != LPB_OK) { c->xs.clear(); c->ys.clear(); c->zs.clear(); }
    return st;
}

lpb_status lpb_evaluate_batch(lpb_ctx* c, int n_sys, const double* const* q, double* const* phi, int on_device)
{
    if (!c) return LPB_EINVAL;
    if (!c->batched || !c->have_tree) return fail(c, LPB_ESTATE, "lpb_set_systems and lpb_build_trees must come first");
    if (n_sys != c->plan.nsys || !q || !phi) return fail(c, LPB_EINVAL, "bad system arrays");
    return evaluate_common(c, n_sys, q, phi, on_device);
}

lpb_status lpb_get_stats(const lpb_ctx* c, lpb_stats* stats)
{
    if (!c || !stats) return LPB_EINVAL;
    *stats = c->stats;
    return LPB_OK;
}

lpb_status lpb_fmm_info(const lpb_ctx* c, int sys, int fmm, int* desc, double* root, int64_t* nt, int64_t* ns,
                        uint64_t* tkeys, uint64_t* skeys)
{
    if (!c) return LPB_EINVAL;
    const Plan& P = c->plan;
    if (!c->have_tree || sys < 0 || sys >= P.nsys) return LPB_EINVAL;
    // FMMs of this system in plan order
    int k = -1, found = -1;
    for (size_t i = 0; i < P.fmm.size(); ++i)
        if (P.fmm[i].sys == sys && ++k == fmm) {
            found = (int)i;
            break;
        }
    if (found < 0) return LPB_EINVAL;
    const FmmDesc& F = P.fmm[found];
    if (desc) {
        desc[0] = F.kind; desc[1] = F.l; desc[2] = F.lp; desc[3] = F.a; desc[4] = F.b; desc[5] = F.H;
    }
    if (root) { root[0] = F.cx; root[1] = F.cy; root[2] = F.cz; root[3] = F.R; }
    if (nt) *nt = F.ntgt;
    if (ns) *ns = F.nsrc;
    // leaf keys of the points of this FMM's trees (leaves are contiguous per
    // tree), in the FMM's original orientation, ordered by charge index
    // (the charge indices of the tree's points come from the device)
    auto gather = [&](const TreeDesc& T, const std::vector<int>& lstart, const int* dcidx,
                      const std::vector<uint64_t>& lcell, const std::vector<int>& llv, uint64_t* out) {
        if (T.nleaf == 0) return true;
        const int p0 = lstart[T.leaf0], p1 = lstart[T.leaf0 + T.nleaf];
        std::vector<int> cidx(p1 - p0);
        if (hipMemcpy(cidx.data(), dcidx + p0, cidx.size() * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return false;
        std::vector<std::pair<int, uint64_t>> v;
        for (int l = T.leaf0; l < T.leaf0 + T.nleaf; ++l)
            for (int j = lstart[l]; j < lstart[l + 1]; ++j) {
                const uint64_t key = P.adaptive ? leaf_key(lcell[l], llv[l], F.flip) | ((uint64_t)llv[l] << 58)
                                                : leaf_key(lcell[l], F.H, F.flip);
                v.push_back({cidx[j - p0], key});
            }
        std::sort(v.begin(), v.end());
        for (size_t i = 0; i < v.size(); ++i) out[i] = v[i].second;
        return true;
    };
    const bool mixed = c->opt.precision == LPB_MIXED;
    if (tkeys && !gather(P.trees[F.tgt_tree], P.tl_start, mixed ? c->a32.t_cidx : c->a64.t_cidx, P.tl_cell, P.tl_lv, tkeys))
        return LPB_EDEVICE;
    if (skeys && !gather(P.trees[F.src_tree], P.sl_start, mixed ? c->a32.s_cidx : c->a64.s_cidx, P.sl_cell, P.sl_lv, skeys))
        return LPB_EDEVICE;
    return LPB_OK;
}

lpb_status lpb_debug_parts(const lpb_ctx* c, double* out, int* nslots)
{
    if (!c || !nslots) return LPB_EINVAL;
    *nslots = c->plan.nslots;
    if (!out || !c->have_tree) return LPB_OK;
    const double* parts = (c->opt.precision == LPB_MIXED) ? c->a32.parts : c->a64.parts;
    const size_t nc = (size_t)c->plan.ncharges, n = (size_t)c->plan.nslots * nc;
    if (!n) return LPB_OK;
    if (hipMemcpy(out, parts, n * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) return LPB_EDEVICE;
    // the free-space near field's own slot, added to slot 0
    std::vector<double> near(nc);
    if (hipMemcpy(near.data(), parts + n, nc * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) return LPB_EDEVICE;
    for (size_t i = 0; i < nc; ++i) out[i] += near[i];
    return LPB_OK;
}

const char* lpb_last_error(const lpb_ctx* c)
{
    if (!c) return g_create_error.c_str();
    return c->err.c_str();
}

void lpb_destroy(lpb_ctx* c)
{
    if (!c) return;
    (void)hipSetDevice(c->opt.device);
    (void)hipDeviceSynchronize();
    drop_graph(c);
    free_bufs(c, c->plan_bufs);
    free_bufs(c, c->op_bufs);
    for (DevBuf* b : {&c->d_btab, &c->d_gtab, &c->d_glx, &c->d_glw, &c->d_flag}) free_buf(c, *b);
    if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
    if (c->fork.side) (void)hipStreamDestroy(c->fork.side);
    if (c->fork.fork) (void)hipEventDestroy(c->fork.fork);
    if (c->fork.join) (void)hipEventDestroy(c->fork.join);
    if (c->fork.near) (void)hipStreamDestroy(c->fork.near);
    if (c->fork.near_fork) (void)hipEventDestroy(c->fork.near_fork);
    if (c->fork.near_join) (void)hipEventDestroy(c->fork.near_join);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    for (auto& e : c->evs)
        if (e) (void)hipEventDestroy(e);
    delete c;
}

double lpb_host_gaunt(int n1, int m1, int n2, int m2, int n3, int m3)
{
    if (n1 < 0 || n2 < 0 || n3 < 0 || std::abs(m1) > n1 || std::abs(m2) > n2 || std::abs(m3) > n3) return 0.0;
    return host_gaunt(n1, m1, n2, m2, n3, m3);
}

}  // extern "C"
