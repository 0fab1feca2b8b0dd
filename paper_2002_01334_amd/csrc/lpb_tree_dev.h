// lpb_tree_dev.h -- the per-point part of the plan builder on the GPU.
#pragma once
#include <functional>
#include <string>
#include <vector>

#include "lpb_internal.h"

namespace lpb {

// Every buffer comes from `alloc` and goes back through `free` (the
// context's allocator); kernels and copies run on `stream`.
class DevPointBuilder : public PointBuilder {
public:
    DevPointBuilder(hipStream_t stream, std::function<void*(size_t)> alloc, std::function<void(void*)> free);
    ~DevPointBuilder() override;
    DevPointBuilder(const DevPointBuilder&) = delete;
    DevPointBuilder& operator=(const DevPointBuilder&) = delete;

    // device copies of the coordinates of every system (host arrays)
    bool set_coords(const std::vector<std::vector<double>>& xs, const std::vector<std::vector<double>>& ys,
                    const std::vector<std::vector<double>>& zs, std::string& msg);
    int keys(int sys, int64_t coff, const std::vector<int>& members, const SetFrame& F, double R,
             int counts[kMaxDepth + 1], std::string& msg) override;
    bool leaves(int handle, int H, std::vector<uint64_t>& leaf_key, std::vector<int>& leaf_start,
                std::string& msg) override;
    bool leaves_adaptive(int handle, int cap, bool sep, std::vector<uint64_t>& leaf_key, std::vector<int>& leaf_lv,
                         std::vector<int>& leaf_start, std::string& msg) override;
    int failure() const override { return failure_; }
    // The sets `sets` (in order, n_total points) concatenated into the
    // evaluation arrays: charge index, offsets from the leaf centre (FP32: hi
    // parts in ux.., lo parts in lx..; FP64: lx.. unused) and, when `slot` is
    // given (one per set), the output index slot * ncharges + charge index.
    template <typename T>
    bool gather(const std::vector<int>& sets, const std::vector<int>* slot, int64_t ncharges, int64_t n_total,
                int* cidx, int* out, T* ux, T* uy, T* uz, T* lx, T* ly, T* lz, std::string& msg);

private:
    struct Set {
        int n = 0, H = -1;
        double R = 0.0;
        int64_t coff = 0;
        int* members = nullptr;   // device
        uint64_t* key = nullptr;  // sorted keys
        int* perm = nullptr;      // sorted position -> member position
        double* w = nullptr;      // 3n canonical coordinates, member order
        int* cidx = nullptr;      // sorted charge indices (after leaves)
        double* u = nullptr;      // 3n offsets from the leaf centre, sorted order (after leaves)
    };
    void* get(size_t bytes);
    void put(void*& p);
    // temporaries of one kind, kept and grown from set to set
    enum { kKeyIn, kIdx, kCnt, kSortTmp, kFlag, kPos, kLeafKey, kLeafStart, kScanTmp, kLeafLv, kScratchKinds };
    void* scratch(int kind, size_t bytes);
    void* scr_[kScratchKinds] = {};
    size_t scr_bytes_[kScratchKinds] = {};
    bool check(hipError_t e, const char* what, std::string& msg);
    hipStream_t st_;
    std::function<void*(size_t)> alloc_;
    std::function<void(void*)> free_;
    std::vector<double*> x_, y_, z_;
    std::vector<Set> sets_;
    int failure_ = LPB_EDEVICE;
};

}  // namespace lpb
