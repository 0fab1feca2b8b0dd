// lpb_m2l_tile_kb.h -- the per-offset tiled free-space M2L with the number of
// 16-row blocks fixed at compile time; instantiated for FP64 and FP32 in
// lpb_m2l_tile_kb64.hip and lpb_m2l_tile_kb32.hip.
#pragma once
#include <hip/hip_runtime.h>

#include "lpb_eval_dev.h"

namespace lpb {

// The same product with the number of 16-row blocks KB fixed at compile
// time (p <= 15): the 16-column slabs of the operator stream through a ring
// of D register slabs, so every load is issued D slabs (D * RB * 4 MFMAs)
// ahead of its use, continuing across offsets into the next operator.
// RBW = 0: four waves, each owning ceil(KB/4) row blocks; RBW = 1: KB waves
// of one row block each (more waves per CU to hide latency, same arithmetic
// per output element in the same order, so both give identical results).
template <typename T, int KB, int RBW>
__global__ void __launch_bounds__(RBW == 1 ? 64 * KB : 256) k_m2l_tile_kb(EvalArgs<T> A)
{
    typedef typename Vec4<T>::type V4;
    constexpr int NWT = (RBW == 1) ? KB : 4;              // waves per block
    constexpr int RB = (RBW == 1) ? 1 : (KB + 3) / 4;     // row blocks per wave
    constexpr int NWACT = (KB + RB - 1) / RB;   // waves that own row blocks (the others only gather)
    constexpr int NV = 4 * KB / NWT;                       // staged 4-vectors per thread and offset
    constexpr int D = (RBW == 0 && sizeof(T) == 4 && RB <= 2) ? ((KB % 4 == 0) ? 4 : ((KB % 2 == 0) ? 2 : 1))
                                                               : ((KB % 2 == 0) ? 2 : 1);
    constexpr int NT = 64, CB = 4, KP = 16 * KB;
    constexpr int NTP = NT + (sizeof(T) == 4 ? 16 : 8);   // padded LDS row (bank spread)
    extern __shared__ unsigned char smem_raw[];
    T* Bs = reinterpret_cast<T*>(smem_raw);               // [KP][NTP]
    __shared__ int s_le[NT];
    const int K = A.K;
    const Tile tile = A.tiles[sched_index(blockIdx.x, gridDim.x, A.tile_sched & 1)];
    const TileFL fl = A.tfl[tile.fl];
    const int nside = fl.nside;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    const int ox = (tile.octant >> 2) & 1, oy = (tile.octant >> 1) & 1, oz = tile.octant & 1;
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
    const int gj = tid / NWT, gpart = tid % NWT;   // column and 4-vector part of the gather
    int gtx, gty, gtz;
    tcoord(gj, gtx, gty, gtz);
    const bool gvalid = s_le[gj] >= 0;
    const int* codes = A.oct_codes + tile.octant * kVOffsets;
    V4 greg[NV];
    auto fetch = [&](int d) {
        const int code = codes[d];
        const int sx = gtx + code / 49 - 3, sy = gty + (code / 7) % 7 - 3, sz = gtz + code % 7 - 3;
        int me = -1;
        if (gvalid && sx >= 0 && sy >= 0 && sz >= 0 && sx < nside && sy < nside && sz < nside)
            me = A.grid_me[fl.grid_off + ((size_t)sx * nside + sy) * nside + sz];
        // a missing source reads the zero row
        const T* src = A.me + (size_t)(me < 0 ? A.n_me : me) * KP + 4 * gpart;
#pragma unroll
        for (int i = 0; i < NV; ++i) greg[i] = *reinterpret_cast<const V4*>(src + 4 * NWT * i);
    };
    auto opent = [&](int d) { return A.optab[fl.optab_off + codes[d]]; };
    auto opA = [&](int d) {
        return A.pool_swz + (size_t)A.swz_index[opent(d) & ((1 << kReflShift) - 1)] * KP * KP;
    };
    V4 ring[D][RB];
    // row blocks past KB (last active wave only) repeat the last block; their
    // rows are >= K and never stored
    auto loadA = [&](const T* Aw, int s4, V4 (&dst)[RB]) {
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            const int rbg = min(w * RB + rb, KB - 1);
            dst[rb] = *reinterpret_cast<const V4*>(Aw + (((size_t)rbg * KB + s4) * 64 + l) * 4);
        }
    };
    const T* Aw = opA(0);
    if (w < NWACT) {
#pragma unroll
        for (int i = 0; i < D; ++i) loadA(Aw, i, ring[i]);
    }
    fetch(0);
    // products of up to GRP consecutive offsets of one reflection class chain in
    // the MFMA accumulators; the row signs and the compensated sum follow per run
    constexpr int GRP = (sizeof(T) == 4) ? 4 : 1;
    int run = 0;
    for (int d = 0; d < kVOffsets; ++d) {
        const int cls = opent(d) >> kReflShift;
        const T* sg = A.refl_sign + (size_t)cls * KP;
        __syncthreads();   // every wave is done with the previous offset's B
#pragma unroll
        for (int i = 0; i < NV; ++i) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int k = 4 * (NWT * i + gpart) + e;
                Bs[k * NTP + gj] = greg[i][e] * sg[k];
            }
        }
        __syncthreads();
        const bool more = d + 1 < kVOffsets;
        const T* Awn = more ? opA(d + 1) : Aw;
        if (more) fetch(d + 1);   // next offset's sources load during this offset's products
        const bool flush = !more || run + 1 == GRP || (opent(d + 1) >> kReflShift) != cls;
        if (w < NWACT) {          // wave-uniform; the product loop itself has no branches
            if (run == 0) {
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = V4{0, 0, 0, 0};
            }
#pragma unroll
            for (int s4 = 0; s4 < KB; ++s4) {
                V4 a4[RB];
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) a4[rb] = ring[s4 % D][rb];
                if (s4 + D < KB) loadA(Aw, s4 + D, ring[s4 % D]);
                else loadA(Awn, s4 + D - KB, ring[s4 % D]);   // (the last offset reloads its own operator)
#pragma unroll
                for (int ss = 0; ss < 4; ++ss) {
                    const int kk = 16 * s4 + 4 * ss + (l >> 4);
                    T b[CB];
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb) b[cb] = Bs[kk * NTP + cb * 16 + (l & 15)];
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                        for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = mfma16(a4[rb][ss], b[cb], acc[rb][cb]);
                }
            }
            if (flush) {
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
        }
        run = flush ? 0 : run + 1;
        Aw = Awn;
    }
    if (w >= NWACT) return;
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

// Launch the fixed-KB kernel for the expansion stride of A; false if KB has
// no specialisation for T (FP64 above 12 blocks would spill registers).
template <typename T>
bool launch_m2l_tile_kb(const EvalArgs<T>& A, bool wide, hipStream_t st)
{
    const int KB = A.KP / 16;
    const size_t sm = sizeof(T) * (size_t)A.KP * (64 + (sizeof(T) == 4 ? 16 : 8));
    dim3 g(A.n_tiles), b(256);
#define LPB_TKB(N)                                                                                  \
    case N:                                                                                         \
        if (wide) hipLaunchKernelGGL((k_m2l_tile_kb<T, N, 1>), g, dim3(64 * N), sm, st, A);         \
        else hipLaunchKernelGGL((k_m2l_tile_kb<T, N, 0>), g, b, sm, st, A);                         \
        return true;
    switch (KB) {
        LPB_TKB(1) LPB_TKB(2) LPB_TKB(3) LPB_TKB(4) LPB_TKB(5) LPB_TKB(6)
        LPB_TKB(7) LPB_TKB(8) LPB_TKB(9) LPB_TKB(10) LPB_TKB(11) LPB_TKB(12)
    default: break;
    }
    if constexpr (sizeof(T) == 4) {
        switch (KB) {
            LPB_TKB(13) LPB_TKB(14) LPB_TKB(15) LPB_TKB(16)
        default: break;
        }
    }
#undef LPB_TKB
    return false;
}

}  // namespace lpb
