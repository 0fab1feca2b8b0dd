// lpb_m2l_tile.hip -- tiled free-space M2L on the matrix cores (eq. metole at
// tree levels 4..8): the generic per-offset product and the launcher that
// picks among the forms (orbit form: lpb_m2l_orbit.h; per-offset products
// with KB fixed at compile time: lpb_m2l_tile_kb.h).
#include <hip/hip_runtime.h>

#include "lpb_eval_dev.h"

namespace lpb {

template <typename T, int RB>
__global__ void __launch_bounds__(256) k_m2l_tile(EvalArgs<T> A)
{
    typedef typename Vec4<T>::type V4;
    constexpr int NT = 64, CB = 4, GMAX = 4 * RB;
    constexpr int NTP = NT + (sizeof(T) == 4 ? 16 : 8);   // padded LDS row (bank spread)
    extern __shared__ unsigned char smem_raw[];
    T* Bs = reinterpret_cast<T*>(smem_raw);               // [KP][NTP]
    __shared__ int s_le[NT];
    const int K = A.K, KP = A.KP, KB = KP / 16;
    const Tile tile = A.tiles[sched_index(blockIdx.x, gridDim.x, A.tile_sched & 1)];
    const TileFL fl = A.tfl[tile.fl];
    const int nside = fl.nside;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    const int ox = (tile.octant >> 2) & 1, oy = (tile.octant >> 1) & 1, oz = tile.octant & 1;
    // per-offset products accumulate in `acc`; the sum over the 189 offsets is
    // compensated (Kahan, FP32) in `tot`/`cmp`, which keeps the FP32 error at the
    // level of a single offset's product
    V4 acc[RB][CB], tot[RB][CB], cmp[RB][CB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) tot[rb][cb] = cmp[rb][cb] = V4{0, 0, 0, 0};
    auto tcoord = [&](int j, int& tx, int& ty, int& tz) {
        tx = 2 * (tile.px0 + (j >> 4)) + ox;
        ty = 2 * (tile.py0 + ((j >> 2) & 3)) + oy;
        tz = 2 * (tile.pz0 + (j & 3)) + oz;
    };
    if (tid < NT) {
        int tx, ty, tz;
        tcoord(tid, tx, ty, tz);
        s_le[tid] = (tx < nside && ty < nside && tz < nside)
                        ? A.grid_le[fl.grid_off + ((size_t)tx * nside + ty) * nside + tz] : -1;
    }
    __syncthreads();
    // gather role of this thread: target column gj, rows 16 i + 4 gpart .. +3
    const int gj = tid >> 2, gpart = tid & 3;
    int gtx, gty, gtz;
    tcoord(gj, gtx, gty, gtz);
    const bool gvalid = s_le[gj] >= 0;
    const int* codes = A.oct_codes + tile.octant * kVOffsets;
    V4 greg[GMAX];
    auto fetch = [&](int d) {
        const int code = codes[d];
        const int sx = gtx + code / 49 - 3, sy = gty + (code / 7) % 7 - 3, sz = gtz + code % 7 - 3;
        int me = -1;
        if (gvalid && sx >= 0 && sy >= 0 && sz >= 0 && sx < nside && sy < nside && sz < nside)
            me = A.grid_me[fl.grid_off + ((size_t)sx * nside + sy) * nside + sz];
        const T* src = A.me + (size_t)(me < 0 ? 0 : me) * KP + 4 * gpart;
#pragma unroll
        for (int i = 0; i < GMAX; ++i)
            greg[i] = (me >= 0 && i < KB) ? *reinterpret_cast<const V4*>(src + 16 * i) : V4{0, 0, 0, 0};
    };
    fetch(0);
    for (int d = 0; d < kVOffsets; ++d) {
        __syncthreads();   // every wave is done with the previous offset's B
        const int ent = A.optab[fl.optab_off + codes[d]];
        const int op = ent & ((1 << kReflShift) - 1);
        const T* sg = A.refl_sign + (size_t)(ent >> kReflShift) * KP;
#pragma unroll
        for (int i = 0; i < GMAX; ++i) {
            if (i < KB) {
#pragma unroll
                for (int e = 0; e < 4; ++e) Bs[(16 * i + 4 * gpart + e) * NTP + gj] = greg[i][e] * sg[16 * i + 4 * gpart + e];
            }
        }
        __syncthreads();
        if (d + 1 < kVOffsets) fetch(d + 1);   // next offset's sources load during this offset's products
        const T* Aw = A.pool_swz + (size_t)A.swz_index[op] * KP * KP;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = V4{0, 0, 0, 0};
        V4 an[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            int rbg = w * RB + rb;
            an[rb] = (rbg < KB) ? *reinterpret_cast<const V4*>(Aw + ((size_t)rbg * KB * 64 + l) * 4) : V4{0, 0, 0, 0};
        }
        for (int s4 = 0; s4 < KB; ++s4) {
            V4 a4[RB];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                a4[rb] = an[rb];
                int rbg = w * RB + rb;
                if (rbg < KB && s4 + 1 < KB)
                    an[rb] = *reinterpret_cast<const V4*>(Aw + (((size_t)rbg * KB + s4 + 1) * 64 + l) * 4);
            }
#pragma unroll
            for (int ss = 0; ss < 4; ++ss) {
                const int kk = 16 * s4 + 4 * ss + (l >> 4);
                T b[CB];
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) b[cb] = Bs[kk * NTP + cb * 16 + (l & 15)];
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    if (w * RB + rb < KB) {
#pragma unroll
                        for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = mfma16(a4[rb][ss], b[cb], acc[rb][cb]);
                    }
                }
            }
        }
        // result rows: the second sign flip of D A D
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            V4 sr;
#pragma unroll
            for (int r = 0; r < 4; ++r) sr[r] = sg[min(w * RB + rb, KB - 1) * 16 + mfma_row(T(0), l, r)];
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) acc[rb][cb] *= sr;
        }
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                if (sizeof(T) == 4) {
                    V4 y = acc[rb][cb] - cmp[rb][cb];
                    V4 t = tot[rb][cb] + y;
                    cmp[rb][cb] = (t - tot[rb][cb]) - y;
                    tot[rb][cb] = t;
                } else {
                    tot[rb][cb] += acc[rb][cb];
                }
            }
    }
    // accumulate into the local expansions
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        int rbg = w * RB + rb;
        if (rbg >= KB) continue;
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            int j = cb * 16 + (l & 15);
            int le = s_le[j];
            if (le < 0) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int row = rbg * 16 + mfma_row(T(0), l, r);
                if (row < K) A.le[(size_t)le * KP + row] += tot[rb][cb][r];
            }
        }
    }
}

template <typename T>
void launch_m2l_tile(const EvalArgs<T>& A, hipStream_t st)
{
    const int KB = A.KP / 16, RB = (KB + 3) / 4;
    const size_t sm = sizeof(T) * (size_t)A.KP * (64 + (sizeof(T) == 4 ? 16 : 8));
    dim3 g(A.n_tiles), b(256);
    // variant bit of the schedule: KB waves of one row block each
    const bool wide = (A.tile_sched >> 1) & 1;
    if constexpr (sizeof(T) == 4) {
        // (row byte offsets of the expansions are 32-bit in the orbit kernel;
        // schedule bit 2 asks for the per-offset form instead)
        if (A.pool_orb && A.p >= kOrbitMinP && A.p <= kOrbitMaxP && !((A.tile_sched >> 2) & 1) &&
            (size_t)(A.n_me + 1) * A.KP * sizeof(float) < ((size_t)1 << 32)) {
#define LPB_ORB(PP) \
    case PP: launch_m2l_orbit_p<PP>(A, st); return;
            switch (A.p) {
                LPB_ORB(5) LPB_ORB(6) LPB_ORB(7) LPB_ORB(8) LPB_ORB(9) LPB_ORB(10)
                LPB_ORB(11) LPB_ORB(12) LPB_ORB(13) LPB_ORB(14) LPB_ORB(15)
            default: break;
            }
#undef LPB_ORB
        }
    }
    if (launch_m2l_tile_kb<T>(A, wide, st)) return;
    switch (RB) {
    case 1: hipLaunchKernelGGL((k_m2l_tile<T, 1>), g, b, sm, st, A); break;
    case 2: hipLaunchKernelGGL((k_m2l_tile<T, 2>), g, b, sm, st, A); break;
    case 3: hipLaunchKernelGGL((k_m2l_tile<T, 3>), g, b, sm, st, A); break;
    case 4: hipLaunchKernelGGL((k_m2l_tile<T, 4>), g, b, sm, st, A); break;
    case 5: hipLaunchKernelGGL((k_m2l_tile<T, 5>), g, b, sm, st, A); break;
    case 6: hipLaunchKernelGGL((k_m2l_tile<T, 6>), g, b, sm, st, A); break;
    default: hipLaunchKernelGGL((k_m2l_tile<T, 7>), g, b, sm, st, A); break;
    }
}

template void launch_m2l_tile<double>(const EvalArgs<double>&, hipStream_t);
template void launch_m2l_tile<float>(const EvalArgs<float>&, hipStream_t);

}  // namespace lpb
