// lpb_tree_dev.hip -- the per-point part of the plan builder on the GPU: the
// canonical coordinates, fine cells and Morton keys of each point set, their
// stable radix sort, the distinct cells per level (the depth rule), the
// leaves, and every point's offset from its leaf centre.  The arithmetic is
// the host rule's, operation for operation (no contraction), so the plan is
// the same whichever side builds it:
//   fine cell per axis: floor((w + R) / (2R) * 65536) clamped to [0, 65535];
//   key: the fine cells' bits interleaved x, y, z from the top down;
//   leaf centre: -R + (i + 0.5) (2R / 2^H) per axis.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "lpb_tree_dev.h"

namespace lpb {

namespace {

__device__ inline uint32_t fine_cell_dev(double w, double R)
{
#pragma clang fp contract(off)
    const double t = (w + R) / (2.0 * R);
    double f = floor(t * 65536.0);
    if (!(f >= 0.0)) f = 0.0;
    if (f > 65535.0) f = 65535.0;
    return (uint32_t)f;
}

__device__ inline uint64_t spread3_dev(uint32_t v)
{
    uint64_t x = v & 0xffffu;
    x = (x | (x << 16)) & 0x0000ff0000ffull;
    x = (x | (x << 8)) & 0x00f00f00f00full;
    x = (x | (x << 4)) & 0x0c30c30c30c3ull;
    x = (x | (x << 2)) & 0x249249249249ull;
    return x;
}

__device__ inline uint32_t compact3_dev(uint64_t x)
{
    x &= 0x249249249249ull;
    x = (x | (x >> 2)) & 0x0c30c30c30c3ull;
    x = (x | (x >> 4)) & 0x00f00f00f00full;
    x = (x | (x >> 8)) & 0x0000ff0000ffull;
    x = (x | (x >> 16)) & 0xffffull;
    return (uint32_t)x;
}

// canonical coordinates and fine-cell key of every member
__global__ void k_set_keys(int n, const int* __restrict__ mem, const double* __restrict__ x,
                           const double* __restrict__ y, const double* __restrict__ z, SetFrame F, double R,
                           uint64_t* __restrict__ key, int* __restrict__ idx, double* __restrict__ w)
{
#pragma clang fp contract(off)
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int m = mem[i];
    const double w0 = x[m] - F.ax, w1 = y[m] - F.ay;
    double w2;
    if (F.mode == 0) {
        w2 = z[m] - F.az;
    } else {
        const double t = F.side == 1 ? z[m] - F.az : F.az - z[m];
        w2 = F.target ? t : -t;
    }
    w[i] = w0;
    w[(size_t)n + i] = w1;
    w[2 * (size_t)n + i] = w2;
    key[i] = (spread3_dev(fine_cell_dev(w0, R)) << 2) | (spread3_dev(fine_cell_dev(w1, R)) << 1) |
             spread3_dev(fine_cell_dev(w2, R));
    idx[i] = i;
}

// distinct level-l cells of the sorted keys, l = 0..kMaxDepth (one count per
// wave and level, then one atomic add)
__global__ void __launch_bounds__(256) k_level_counts(int n, const uint64_t* __restrict__ key, int* __restrict__ counts)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t k = i < n ? key[i] : 0, kp = (i > 0 && i < n) ? key[i - 1] : 0;
    for (int lv = 0; lv <= kMaxDepth; ++lv) {
        const int sh = 3 * (kCellBits - lv);
        const bool first = i < n && (i == 0 || (k >> sh) != (kp >> sh));
        const unsigned long long b = __ballot(first);
        if ((threadIdx.x & 63) == 0 && b) atomicAdd(&counts[lv], __popcll(b));
    }
}

// 1 where a point starts a level-H cell
__global__ void k_leaf_flags(int n, const uint64_t* __restrict__ key, int H, int* __restrict__ flag)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int sh = 3 * (kCellBits - H);
    flag[i] = (i == 0 || (key[i] >> sh) != (key[i - 1] >> sh)) ? 1 : 0;
}

// leaf keys and starts (pos: inclusive scan of the flags), and every point's
// charge index and offset from its leaf centre in sorted order
__global__ void k_leaf_points(int n, const uint64_t* __restrict__ key, const int* __restrict__ flag,
                              const int* __restrict__ pos, const int* __restrict__ perm, const int* __restrict__ mem,
                              int64_t coff, const double* __restrict__ w, int H, double R,
                              uint64_t* __restrict__ lkey, int* __restrict__ lstart, int* __restrict__ cidx,
                              double* __restrict__ u)
{
#pragma clang fp contract(off)
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t k = key[i];
    if (flag[i]) {
        lkey[pos[i] - 1] = k >> (3 * (kCellBits - H));
        lstart[pos[i] - 1] = i;
    }
    const int j = perm[i];
    cidx[i] = (int)(coff + mem[j]);
    const double h = 2.0 * R / (double)(1 << H);
    const int shH = kCellBits - H;
    const uint32_t c[3] = {compact3_dev(k >> 2) >> shH, compact3_dev(k >> 1) >> shH, compact3_dev(k) >> shH};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double ctr = -R + ((int)c[d] + 0.5) * h;
        u[(size_t)d * n + i] = w[(size_t)d * n + j] - ctr;
    }
}

// the same on adaptive leaves: a point's leaf is the last leaf starting at or
// before its sorted position, at that leaf's own level
__global__ void k_leaf_points_adaptive(int n, const uint64_t* __restrict__ key, int nleaf,
                                       const int* __restrict__ lstart, const int* __restrict__ llv,
                                       const int* __restrict__ perm, const int* __restrict__ mem, int64_t coff,
                                       const double* __restrict__ w, double R, int* __restrict__ cidx,
                                       double* __restrict__ u)
{
#pragma clang fp contract(off)
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int lo = 0, hi = nleaf - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (lstart[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    const int H = llv[lo];
    const uint64_t k = key[i];
    const int j = perm[i];
    cidx[i] = (int)(coff + mem[j]);
    const double h = 2.0 * R / (double)(1 << H);
    const int shH = kCellBits - H;
    const uint32_t c[3] = {compact3_dev(k >> 2) >> shH, compact3_dev(k >> 1) >> shH, compact3_dev(k) >> shH};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double ctr = -R + ((int)c[d] + 0.5) * h;
        u[(size_t)d * n + i] = w[(size_t)d * n + j] - ctr;
    }
}

// one set's points into the evaluation arrays at offset g0
template <typename T>
__global__ void k_gather_points(int n, int64_t g0, const int* __restrict__ cidx, const double* __restrict__ u, int slot,
                                int64_t ncharges, int* __restrict__ ocidx, int* __restrict__ oout, T* __restrict__ ux,
                                T* __restrict__ uy, T* __restrict__ uz, T* __restrict__ lx, T* __restrict__ ly,
                                T* __restrict__ lz)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t o = g0 + i;
    const int ci = cidx[i];
    ocidx[o] = ci;
    if (oout) oout[o] = (int)(slot * ncharges + ci);
    T* hi[3] = {ux, uy, uz};
    T* lo[3] = {lx, ly, lz};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        // FP32: hi = (float)u and lo = (float)(u - hi), so hi + lo carries u to ~2^-48 relative
        const double v = u[(size_t)d * n + i];
        const T h = (T)v;
        hi[d][o] = h;
        if (sizeof(T) == 4) lo[d][o] = (T)(v - (double)h);
    }
}

inline unsigned nblk(int n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

DevPointBuilder::DevPointBuilder(hipStream_t stream, std::function<void*(size_t)> alloc, std::function<void(void*)> free)
    : st_(stream), alloc_(std::move(alloc)), free_(std::move(free))
{
}

DevPointBuilder::~DevPointBuilder()
{
    (void)hipStreamSynchronize(st_);
    for (auto& s : sets_) {
        void* p[] = {s.members, s.key, s.perm, s.w, s.cidx, s.u};
        for (void* q : p)
            if (q) free_(q);
    }
    for (auto* v : {&x_, &y_, &z_})
        for (double* q : *v)
            if (q) free_(q);
    for (void* q : scr_)
        if (q) free_(q);
}

void* DevPointBuilder::scratch(int kind, size_t bytes)
{
    if (scr_[kind] && scr_bytes_[kind] >= bytes) return scr_[kind];
    if (scr_[kind]) {
        (void)hipStreamSynchronize(st_);   // (nothing in flight may still use it)
        free_(scr_[kind]);
    }
    bytes = std::max<size_t>(bytes, 4096);
    scr_[kind] = get(bytes);
    scr_bytes_[kind] = scr_[kind] ? bytes : 0;
    return scr_[kind];
}

void* DevPointBuilder::get(size_t bytes)
{
    void* p = alloc_(std::max<size_t>(bytes, 8));
    if (!p) failure_ = LPB_ENOMEM;
    return p;
}

void DevPointBuilder::put(void*& p)
{
    if (p) free_(p);
    p = nullptr;
}

bool DevPointBuilder::check(hipError_t e, const char* what, std::string& msg)
{
    if (e == hipSuccess) return true;
    failure_ = e == hipErrorOutOfMemory ? LPB_ENOMEM : LPB_EDEVICE;
    msg = std::string("point builder, ") + what + ": " + hipGetErrorString(e);
    return false;
}

bool DevPointBuilder::set_coords(const std::vector<std::vector<double>>& xs, const std::vector<std::vector<double>>& ys,
                                 const std::vector<std::vector<double>>& zs, std::string& msg)
{
    for (size_t s = 0; s < xs.size(); ++s) {
        const size_t n = xs[s].size();
        const std::vector<double>* src[3] = {&xs[s], &ys[s], &zs[s]};
        std::vector<double*>* dst[3] = {&x_, &y_, &z_};
        for (int d = 0; d < 3; ++d) {
            double* p = (double*)get(n * sizeof(double));
            dst[d]->push_back(p);
            if (!p) {
                msg = "point builder: device allocation failed";
                return false;
            }
            if (n && !check(hipMemcpyAsync(p, src[d]->data(), n * sizeof(double), hipMemcpyHostToDevice, st_),
                            "coordinate upload", msg))
                return false;
        }
    }
    return check(hipStreamSynchronize(st_), "coordinate upload", msg);
}

int DevPointBuilder::keys(int sys, int64_t coff, const std::vector<int>& members, const SetFrame& F, double R,
                          int counts[kMaxDepth + 1], std::string& msg)
{
    Set S;
    S.n = (int)members.size();
    S.R = R;
    S.coff = coff;
    const int n = S.n;
    sets_.push_back(S);
    Set& s = sets_.back();
    const int handle = (int)sets_.size() - 1;
    s.members = (int*)get(n * sizeof(int));
    s.key = (uint64_t*)get(n * sizeof(uint64_t));
    s.perm = (int*)get(n * sizeof(int));
    s.w = (double*)get(3 * (size_t)n * sizeof(double));
    uint64_t* kin = (uint64_t*)scratch(kKeyIn, n * sizeof(uint64_t));
    int* idx = (int*)scratch(kIdx, n * sizeof(int));
    int* cnt = (int*)scratch(kCnt, (kMaxDepth + 1) * sizeof(int));
    void* tmp = nullptr;
    bool ok = s.members && s.key && s.perm && s.w && kin && idx && cnt;
    if (!ok) msg = "point builder: device allocation failed";
    size_t tb = 0;
    if (ok && n > 0) {
        ok = check(hipMemcpyAsync(s.members, members.data(), n * sizeof(int), hipMemcpyHostToDevice, st_),
                   "member upload", msg);
        if (ok) {
            hipLaunchKernelGGL(k_set_keys, dim3(nblk(n, 256)), dim3(256), 0, st_, n, s.members, x_[sys], y_[sys],
                               z_[sys], F, R, kin, idx, s.w);
            ok = check(hipGetLastError(), "key kernel", msg);
        }
        // a stable LSD sort of the 48-bit keys: equal keys keep member (charge) order
        if (ok) ok = check(rocprim::radix_sort_pairs(nullptr, tb, kin, s.key, idx, s.perm, (unsigned)n, 0, 48, st_),
                           "sort size", msg);
        if (ok) {
            tmp = scratch(kSortTmp, tb);
            if (!tmp) {
                ok = false;
                msg = "point builder: device allocation failed";
            }
        }
        if (ok) ok = check(rocprim::radix_sort_pairs(tmp, tb, kin, s.key, idx, s.perm, (unsigned)n, 0, 48, st_), "sort",
                           msg);
    }
    if (ok) ok = check(hipMemsetAsync(cnt, 0, (kMaxDepth + 1) * sizeof(int), st_), "count clear", msg);
    if (ok && n > 0) {
        hipLaunchKernelGGL(k_level_counts, dim3(nblk(n, 256)), dim3(256), 0, st_, n, s.key, cnt);
        ok = check(hipGetLastError(), "count kernel", msg);
    }
    if (ok) ok = check(hipMemcpyAsync(counts, cnt, (kMaxDepth + 1) * sizeof(int), hipMemcpyDeviceToHost, st_),
                       "count download", msg);
    if (ok) ok = check(hipStreamSynchronize(st_), "keys", msg);
    return ok ? handle : -1;
}

bool DevPointBuilder::leaves(int handle, int H, std::vector<uint64_t>& leaf_key, std::vector<int>& leaf_start,
                             std::string& msg)
{
    Set& s = sets_[handle];
    const int n = s.n;
    s.H = H;
    leaf_key.clear();
    leaf_start.clear();
    if (n == 0) return true;
    int* flag = (int*)scratch(kFlag, n * sizeof(int));
    int* pos = (int*)scratch(kPos, n * sizeof(int));
    uint64_t* lk = (uint64_t*)scratch(kLeafKey, n * sizeof(uint64_t));
    int* ls = (int*)scratch(kLeafStart, n * sizeof(int));
    s.cidx = (int*)get(n * sizeof(int));
    s.u = (double*)get(3 * (size_t)n * sizeof(double));
    void* tmp = nullptr;
    size_t tb = 0;
    int nleaf = 0;
    bool ok = flag && pos && lk && ls && s.cidx && s.u;
    if (!ok) msg = "point builder: device allocation failed";
    if (ok) {
        hipLaunchKernelGGL(k_leaf_flags, dim3(nblk(n, 256)), dim3(256), 0, st_, n, s.key, H, flag);
        ok = check(hipGetLastError(), "leaf kernel", msg);
    }
    if (ok) ok = check(rocprim::inclusive_scan(nullptr, tb, flag, pos, (size_t)n, rocprim::plus<int>(), st_), "scan size",
                       msg);
    if (ok) {
        tmp = scratch(kScanTmp, tb);
        if (!tmp) {
            ok = false;
            msg = "point builder: device allocation failed";
        }
    }
    if (ok) ok = check(rocprim::inclusive_scan(tmp, tb, flag, pos, (size_t)n, rocprim::plus<int>(), st_), "scan", msg);
    if (ok) {
        hipLaunchKernelGGL(k_leaf_points, dim3(nblk(n, 256)), dim3(256), 0, st_, n, s.key, flag, pos, s.perm, s.members,
                           s.coff, s.w, H, s.R, lk, ls, s.cidx, s.u);
        ok = check(hipGetLastError(), "leaf point kernel", msg);
    }
    if (ok) ok = check(hipMemcpyAsync(&nleaf, pos + (n - 1), sizeof(int), hipMemcpyDeviceToHost, st_), "leaf count", msg);
    if (ok) ok = check(hipStreamSynchronize(st_), "leaves", msg);
    if (ok) {
        leaf_key.resize(nleaf);
        leaf_start.resize(nleaf);
        ok = check(hipMemcpyAsync(leaf_key.data(), lk, nleaf * sizeof(uint64_t), hipMemcpyDeviceToHost, st_),
                   "leaf download", msg) &&
             check(hipMemcpyAsync(leaf_start.data(), ls, nleaf * sizeof(int), hipMemcpyDeviceToHost, st_),
                   "leaf download", msg) &&
             check(hipStreamSynchronize(st_), "leaves", msg);
    }
    // the sort state is no longer needed
    void* d[] = {s.key, s.perm, s.w, s.members};
    for (void*& q : d) put(q);
    s.key = nullptr;
    s.perm = nullptr;
    s.w = nullptr;
    s.members = nullptr;
    return ok;
}

bool DevPointBuilder::leaves_adaptive(int handle, int cap, bool sep, std::vector<uint64_t>& leaf_key,
                                      std::vector<int>& leaf_lv, std::vector<int>& leaf_start, std::string& msg)
{
    Set& s = sets_[handle];
    const int n = s.n;
    leaf_key.clear();
    leaf_lv.clear();
    leaf_start.clear();
    if (n == 0) return true;
    std::vector<uint64_t> k(n);
    if (!check(hipMemcpyAsync(k.data(), s.key, n * sizeof(uint64_t), hipMemcpyDeviceToHost, st_), "key download", msg) ||
        !check(hipStreamSynchronize(st_), "key download", msg))
        return false;
    // divide from the root down (above kMaxDepth) a box of more than cap
    // points, and with sep a box that is wider than the distance of its
    // nearest point from the interface plane, up to 3 levels below the level
    // where the occupancy rule stopped (the plane lies between fine cells
    // 32767 and 32768 in z); a divided box is replaced by its non-empty
    // children, in Morton order
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
            leaf_key.push_back(k[a] >> (3 * (kCellBits - lv)));
            leaf_lv.push_back(lv);
            leaf_start.push_back(a);
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
    const int nleaf = (int)leaf_key.size();
    int* ls = (int*)scratch(kLeafStart, nleaf * sizeof(int));
    int* lv = (int*)scratch(kLeafLv, nleaf * sizeof(int));
    s.cidx = (int*)get(n * sizeof(int));
    s.u = (double*)get(3 * (size_t)n * sizeof(double));
    bool ok = ls && lv && s.cidx && s.u;
    if (!ok) msg = "point builder: device allocation failed";
    if (ok)
        ok = check(hipMemcpyAsync(ls, leaf_start.data(), nleaf * sizeof(int), hipMemcpyHostToDevice, st_),
                   "leaf upload", msg) &&
             check(hipMemcpyAsync(lv, leaf_lv.data(), nleaf * sizeof(int), hipMemcpyHostToDevice, st_), "leaf upload",
                   msg);
    if (ok) {
        hipLaunchKernelGGL(k_leaf_points_adaptive, dim3(nblk(n, 256)), dim3(256), 0, st_, n, s.key, nleaf, ls, lv,
                           s.perm, s.members, s.coff, s.w, s.R, s.cidx, s.u);
        ok = check(hipGetLastError(), "leaf point kernel", msg);
    }
    if (ok) ok = check(hipStreamSynchronize(st_), "leaves", msg);
    void* d[] = {s.key, s.perm, s.w, s.members};
    for (void*& q : d) put(q);
    s.key = nullptr;
    s.perm = nullptr;
    s.w = nullptr;
    s.members = nullptr;
    return ok;
}

template <typename T>
bool DevPointBuilder::gather(const std::vector<int>& sets, const std::vector<int>* slot, int64_t ncharges,
                             int64_t n_total, int* cidx, int* out, T* ux, T* uy, T* uz, T* lx, T* ly, T* lz,
                             std::string& msg)
{
    int64_t g0 = 0;
    for (size_t k = 0; k < sets.size(); ++k) {
        const Set& s = sets_[sets[k]];
        if (s.n == 0) continue;
        if (!s.cidx || g0 + s.n > n_total) {
            msg = "point builder: point set without leaves or past the end";
            return false;
        }
        hipLaunchKernelGGL(k_gather_points<T>, dim3(nblk(s.n, 256)), dim3(256), 0, st_, s.n, g0, s.cidx, s.u,
                           slot ? (*slot)[k] : 0, ncharges, cidx, out, ux, uy, uz, lx, ly, lz);
        if (!check(hipGetLastError(), "gather kernel", msg)) return false;
        g0 += s.n;
    }
    if (g0 != n_total) {
        msg = "point builder: point count mismatch";
        return false;
    }
    return check(hipStreamSynchronize(st_), "gather", msg);
}

template bool DevPointBuilder::gather<float>(const std::vector<int>&, const std::vector<int>*, int64_t, int64_t, int*,
                                             int*, float*, float*, float*, float*, float*, float*, std::string&);
template bool DevPointBuilder::gather<double>(const std::vector<int>&, const std::vector<int>*, int64_t, int64_t, int*,
                                              int*, double*, double*, double*, double*, double*, double*, std::string&);

}  // namespace lpb
