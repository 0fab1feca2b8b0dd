// lpb_m2l_orbit.h -- the reflection-orbit form of the tiled free-space M2L
// (FP32, kOrbitMinP <= p <= kOrbitMaxP); each order is instantiated in one of
// the lpb_m2l_orbit_*.hip translation units (they compile in parallel).
#pragma once
#include <hip/hip_runtime.h>

#include "lpb_eval_dev.h"

namespace lpb {


// Tiled M2L by reflection orbits (FP32, p >= kOrbitMinP).  The 189 V-list
// offsets of a child octant fall into 56 orbits {sigma d} of the canonical
// offset d = (|dx|,|dy|,|dz|) under the reflections sigma of the axes, and
// A_{sigma d} = D_sigma A_d D_sigma with D_sigma = diag(chi_sigma(e_k)), e_k the
// sign class of coefficient k and chi_sigma(e) = (-1)^|sigma & e|.  For the
// result rows of class c therefore
//   sum_sigma (D_sigma A_d D_sigma x_sigma)_c = A_d[c, :] B^(c),
//   B^(c) = sum_sigma chi_sigma(c) x'_sigma,   x'_sigma = D_sigma x_sigma:
// one product per orbit instead of one per member.  With the members
// sigma_j = deposit(j, both) | minus (see kOrbits),
//   B^(c) = (-1)^|c & minus| Wc[extract(c, both)],
//   Wc[m] = D_minus sum_j (-1)^|j & m| prod_{axes b of j} D_b x_j,
// a Walsh-Hadamard transform over the nb both-axes whose butterflies carry
// the per-coefficient axis signs (t v for the upper input); the class sign
// (-1)^|c & minus| multiplies the orbit's product before it is added.  The
// operands hold the result rows in class order (orb_rows), so every 16-row
// block has one class.
// Each wave owns 16 targets of the tile (a 16-column block of the product)
// and every row block: per (orbit, 16-coefficient slab) step each lane loads
// four consecutive coefficients of its target's member sources (the B
// operand of four products, the operand layout arranged to match), forms the
// transforms in registers and issues the products; loads run two steps
// ahead.  The orbits come in groups of one both-axes mask (kOrbGroupMask), so
// each gather loads exactly the members its orbit has.  The operator slab of
// a step is the same for the four waves: it is copied once per block into a
// ring of three LDS slots (buffer loads straight to LDS, a barrier per step;
// up to p = 10 two blocks per CU), or, as a tuned alternative, each wave
// gathers it into registers.  Each orbit's products go to the result with
// Kahan compensation.
template <int P, int MASK>
__device__ __forceinline__ void orbit_step(const Vec4<float>::type (&xs)[8], const int __attribute__((ext_vector_type(4))) ek, int minus,
                                           const Vec4<float>::type (&ra)[class_row_blocks(P)],
                                           Vec4<float>::type (&acc)[class_row_blocks(P)])
{
    typedef Vec4<float>::type V4;
    typedef int I4 __attribute__((ext_vector_type(4)));
    constexpr int NRB = class_row_blocks(P);
    constexpr int NB = (MASK & 1) + ((MASK >> 1) & 1) + ((MASK >> 2) & 1);
    constexpr int M = 1 << NB;
    constexpr int AX[3] = {(MASK & 1) ? 0 : ((MASK & 2) ? 1 : 2), (MASK & 1) ? ((MASK & 2) ? 1 : 2) : 2, 2};
    V4 y[M];
#pragma unroll
    for (int j = 0; j < M; ++j) y[j] = xs[j];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        // sign of the 4 coefficients under the reflection of axis AX[b]
        I4 t;
#pragma unroll
        for (int e = 0; e < 4; ++e) t[e] = ((ek[e] >> AX[b]) & 1) << 31;
#pragma unroll
        for (int j = 0; j < M; ++j)
            if (!((j >> b) & 1)) {
                const V4 u = y[j];
                V4 v = y[j | (1 << b)];
#pragma unroll
                for (int e = 0; e < 4; ++e) v[e] = __int_as_float(__float_as_int(v[e]) ^ t[e]);
                y[j] = u + v;
                y[j | (1 << b)] = u - v;
            }
    }
    if (minus) {
        I4 t;
#pragma unroll
        for (int e = 0; e < 4; ++e) t[e] = (__builtin_popcount(ek[e] & minus) & 1) << 31;
#pragma unroll
        for (int j = 0; j < M; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) y[j][e] = __int_as_float(__float_as_int(y[j][e]) ^ t[e]);
    }
    // class c of row block rb reads Wc[extract(c, both)]
    auto ext = [](int c) {
        int m = 0, o = 0;
        for (int bit = 0; bit < 3; ++bit)
            if ((MASK >> bit) & 1) m |= ((c >> bit) & 1) << o++;
        return m;
    };
#pragma unroll
    for (int ss = 0; ss < 4; ++ss)
#pragma unroll
        for (int rb = 0; rb < NRB; ++rb) acc[rb] = mfma16(ra[rb][ss], y[ext(class_of_row_block(P, rb))][ss], acc[rb]);
}

// The operand slab of a step (NRB row blocks of 1 KiB) is staged in LDS and
// shared by the four waves of a block: the slab is read from L2 once per
// block instead of once per wave, and its registers are free.  Up to 9 row
// blocks (p <= 10) two blocks share a CU, so the second block's waves keep the
// matrix cores busy while the first block's waves wait at the per-step
// barrier; above, one block per CU (the accumulators take the registers).
template <int P>
constexpr bool orbit_lds_operands() { return class_row_blocks(P) <= 9; }

// s_waitcnt immediate that waits until at most n vector memory operations are
// outstanding and for every LDS operation (gfx9 encoding: vmcnt low bits
// [3:0], expcnt [6:4] left at its maximum, lgkmcnt [11:8], vmcnt high bits
// [15:14])
constexpr int waitcnt_vm_lgkm0(int n) { return (n & 15) | (7 << 4) | (0 << 8) | ((n >> 4) << 14); }

// LA: operator slabs staged in LDS
template <int P, bool LA>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(LA && orbit_lds_operands<P>() ? 2 : 1)))
k_m2l_orbit(EvalArgs<float> A)
{
    typedef Vec4<float>::type V4;
    constexpr int K = (P + 1) * (P + 1), KB = (K + 15) / 16, KP = 16 * KB;
    constexpr int NRB = class_row_blocks(P);
    constexpr int OPSZ = NRB * KB * 256;     // floats of one operator
    constexpr int NIT = kOrbits * KB;        // steps (even: kOrbits is)
    constexpr int NG = kOrbGrid * kOrbGrid * kOrbGrid;
    constexpr int NLA = (NRB + 3) / 4;       // row blocks each wave stages per step
    constexpr int SLAB = 4 * NLA * 256;      // floats of one staged slab (blocks past NRB unused)
    __shared__ float s_a[LA ? 3 * SLAB : 4]; // ring of three staged slabs
    __shared__ int s_grid[NG];               // ME row of each local source box
    __shared__ int s_tab[kOrbits * kOrbTab]; // the octant's orbit table
    __shared__ int s_kcls[KP];               // sign class of each coefficient
    __shared__ int s_le[64];                 // LE row of each target (-1 none)
    __shared__ int s_aoff[kOrbits];          // operator of each orbit
    const Tile tile = A.tiles[sched_index(blockIdx.x, gridDim.x, A.tile_sched & 1)];
    const TileFL fl = A.tfl[tile.fl];
    const int nside = fl.nside;
    const int tid = threadIdx.x, l = tid & 63;
    const int ox = (tile.octant >> 2) & 1, oy = (tile.octant >> 1) & 1, oz = tile.octant & 1;
    const int* tab = A.orb_tab + tile.octant * (kOrbits * kOrbTab);
    {
        // every gather of the set-up is issued before the first LDS store, so
        // the independent loads are in flight together
        constexpr int NTH = 256, NGL = (NG + NTH - 1) / NTH, NTL = (kOrbits * kOrbTab + NTH - 1) / NTH;
        static_assert(KP <= NTH, "one coefficient class per thread");
        const int gx0 = 2 * tile.px0 + ox - 3, gy0 = 2 * tile.py0 + oy - 3, gz0 = 2 * tile.pz0 + oz - 3;
        int gv[NGL], tv[NTL];
#pragma unroll
        for (int k = 0; k < NGL; ++k) {
            const int i = tid + k * NTH;
            const int sx = gx0 + i / (kOrbGrid * kOrbGrid), sy = gy0 + (i / kOrbGrid) % kOrbGrid, sz = gz0 + i % kOrbGrid;
            gv[k] = -1;
            if (i < NG && sx >= 0 && sy >= 0 && sz >= 0 && sx < nside && sy < nside && sz < nside)
                gv[k] = A.grid_me[fl.grid_off + ((size_t)sx * nside + sy) * nside + sz];
        }
#pragma unroll
        for (int k = 0; k < NTL; ++k) {
            const int i = tid + k * NTH;
            tv[k] = (i < kOrbits * kOrbTab) ? tab[i] : 0;
        }
        const int kv = (tid < KP) ? A.orb_kcls[tid] : 0;
        int lv = -1;
        if (tid < 64) {
            const int tx = 2 * (tile.px0 + (tid >> 4)) + ox, ty = 2 * (tile.py0 + ((tid >> 2) & 3)) + oy,
                      tz = 2 * (tile.pz0 + (tid & 3)) + oz;
            if (tx < nside && ty < nside && tz < nside)
                lv = A.grid_le[fl.grid_off + ((size_t)tx * nside + ty) * nside + tz];
        } else if (tid < 64 + kOrbits) {
            const int q = tid - 64;
            const int op = A.optab[fl.optab_off + tab[q * kOrbTab + 17]] & ((1 << kReflShift) - 1);
            lv = A.orb_index[op];
        }
#pragma unroll
        for (int k = 0; k < NGL; ++k) {
            const int i = tid + k * NTH;
            if (i < NG) s_grid[i] = gv[k] < 0 ? A.n_me : gv[k];   // a missing source reads the zero row
        }
#pragma unroll
        for (int k = 0; k < NTL; ++k) {
            const int i = tid + k * NTH;
            if (i < kOrbits * kOrbTab) s_tab[i] = tv[k];
        }
        if (tid < KP) s_kcls[tid] = kv;
        if (tid < 64) s_le[tid] = lv;
        else if (tid < 64 + kOrbits) s_aoff[tid - 64] = lv;
    }
    __syncthreads();
    const int cb = tid >> 6, g = l >> 4, jj = l & 15, j = 16 * cb + jj;
    const int tli = ((2 * (j >> 4)) * kOrbGrid + 2 * ((j >> 2) & 3)) * kOrbGrid + 2 * (j & 3);
    // the expansions (with the zero row) span under 2^32 bytes: the launch checks it
    const __amdgpu_buffer_rsrc_t rme =
        __builtin_amdgcn_make_buffer_rsrc(A.me, 0, (int)((unsigned)(A.n_me + 1) * (unsigned)(KP * 4)), 0x00020000);
    const unsigned zoff = (unsigned)A.n_me * (unsigned)(KP * 4) + 16u * g;
    // member row byte offsets of the orbit being gathered, its first CNT
    // members: the orbit groups fix the member count at compile time, and the
    // last orbit of a group also gathers the first steps of the next group's
    // first orbit, which has no more members (its absent ones read the zero row)
    // (and the negative one-sign axes of that orbit, in mnext)
    unsigned off[8];
    int mnext = 0;
    auto lorbit = [&](auto cntc, int q) {
        constexpr int CNT = decltype(cntc)::value;
        const int* row = s_tab + q * kOrbTab;
        const int r0 = __builtin_amdgcn_readfirstlane(row[0]);
        const int nm = 1 << (r0 & 15);
        mnext = (r0 >> 7) & 7;
#pragma unroll
        for (int m = 0; m < CNT; ++m)
            off[m] = (m < nm) ? (unsigned)s_grid[tli + row[1 + m]] * (unsigned)(KP * 4) + 16u * g : zoff;
    };
    typedef int I4 __attribute__((ext_vector_type(4)));
    // operand slabs (register path): gathered two steps ahead (DA = 2) while
    // the registers allow, one step ahead for the larger orders (they come
    // mostly from L2)
    constexpr int DA = (LA || NRB > 9) ? 1 : 2;
    V4 xr[2][8], ra[DA][NRB];
    I4 er[2];
    // operand and member gathers are buffer loads: wave-uniform bases and
    // offsets in scalar registers, one fixed 32-bit lane offset, so a gather
    // costs no vector address arithmetic
    const unsigned lane16 = 16u * l;
    auto load_a = [&](int t, V4 (&as)[NRB]) {
        const int q = t / KB, s = t % KB;
        const float* Ao = A.pool_orb + (size_t)__builtin_amdgcn_readfirstlane(s_aoff[q]) * OPSZ;
        const __amdgpu_buffer_rsrc_t ra_ = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(Ao), 0, OPSZ * 4, 0x00020000);
#pragma unroll
        for (int rb = 0; rb < NRB; ++rb)
            as[rb] = __builtin_bit_cast(V4, __builtin_amdgcn_raw_buffer_load_b128(ra_, lane16, (rb * KB + s) * 1024, 0));
    };
    // LDS path: wave cb copies row blocks cb, cb + 4, ... of step t's slab
    // straight into ring slot `slot` (buffer loads to LDS, 16 bytes per lane
    // at 16 l); block numbers past NRB copy block 0 into the unused tail
    auto stage_a = [&](int t, int slot) {
        const int q = t / KB, s = t % KB;
        const float* Ao = A.pool_orb + (size_t)__builtin_amdgcn_readfirstlane(s_aoff[q]) * OPSZ;
        const __amdgpu_buffer_rsrc_t ra_ = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(Ao), 0, OPSZ * 4, 0x00020000);
        float* dst = s_a + slot * SLAB;
#pragma unroll
        for (int i = 0; i < NLA; ++i) {
            const int b = __builtin_amdgcn_readfirstlane(cb + 4 * i);
            const int bs = b < NRB ? b : 0;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(ra_, (__attribute__((address_space(3))) void*)(dst + b * 256), 16,
                                                     lane16, (bs * KB + s) * 1024, 0, 0);
        }
    };
    // gather step t: its first CNT member sources and the coefficient classes
    // (and, with DA = 2, its operand slab)
    auto load = [&](auto cntc, int t, V4 (&xs)[8], V4 (&as)[NRB], I4& ek) {
        constexpr int CNT = decltype(cntc)::value;
        const int s = t % KB;
        if constexpr (!LA) {
            if (s == 0) lorbit(cntc, t / KB);
        }
        if constexpr (DA == 2) load_a(t, as);
#pragma unroll
        for (int m = 0; m < CNT; ++m) xs[m] = __builtin_bit_cast(V4, __builtin_amdgcn_raw_buffer_load_b128(rme, off[m], 64 * s, 0));
        // (LDS path: from global memory, since an LDS read issued after a
        // slab copy would wait for that copy)
        if constexpr (LA) ek = *reinterpret_cast<const I4*>(A.orb_kcls + 16 * s + 4 * g);
        else ek = *reinterpret_cast<const I4*>(s_kcls + 16 * s + 4 * g);
    };
    V4 acc[NRB], tot[NRB], cmp[NRB];
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb) acc[rb] = tot[rb] = cmp[rb] = V4{0, 0, 0, 0};
    typedef std::integral_constant<int, 1 << __builtin_popcount(kOrbGroupMask[0])> NM0;
    if constexpr (LA) {
        lorbit(NM0{}, 0);
        stage_a(0, 0);
    }
    load(NM0{}, 0, xr[0], ra[0], er[0]);
    if constexpr (LA) stage_a(1, 1);
    load(NM0{}, 1, xr[1], ra[DA - 1], er[1]);
    if constexpr (DA == 1 && !LA) load_a(0, ra[0]);
    // LDS path, at step t: wait until step t's slab is in LDS (each step
    // issues NLA slab copies, then NM member gathers and one class load, and
    // the member counts never grow from one orbit group to the next) and
    // every wave is done with slot (t + 2) mod 3 (read at step t - 1); read
    // step t's slab; look up the member rows when step t + 2 starts an orbit
    // (LDS reads go before the next copy is issued: the compiler makes an LDS
    // read wait for every copy to LDS in flight); copy step t + 2's slab
    auto sync_read = [&](auto nmc, int t, V4 (&as)[NRB]) {
        constexpr int NM = decltype(nmc)::value;
        static_assert(NLA + 2 * NM + 2 <= 63, "vmcnt range");
        __builtin_amdgcn_s_waitcnt(waitcnt_vm_lgkm0(NLA + 2 * NM + 2));
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
        const float* src = s_a + (t % 3) * SLAB + 4 * l;
#pragma unroll
        for (int rb = 0; rb < NRB; ++rb) as[rb] = *reinterpret_cast<const V4*>(src + 256 * rb);
        const int tn = min(t + 2, NIT - 1);
        if (tn % KB == 0) lorbit(nmc, tn / KB);
        stage_a(tn, (t + 2) % 3);
    };
    // one orbit: its KB steps with the transform specialised for its both-axes
    // (steps of one orbit form one straight code path, so the transforms of a
    // step can overlap the products of the previous one); step t uses register
    // slot t & 1 and refills it with step t + 2 (the last steps re-gather a
    // valid step)
    auto run = [&](auto maskc, auto parc, int q, int minus) {
        constexpr int MASK = decltype(maskc)::value, PAR = decltype(parc)::value;
        typedef std::integral_constant<int, 1 << __builtin_popcount(MASK)> NM;
        const int t0 = q * KB;
        // (register path: the scheduling fences keep each step's transforms
        // after its own loads' wait: hoisted into the previous step they would
        // wait for the loads just issued; the LDS path's barriers order the
        // steps already)
        constexpr int A0 = (DA == 2) ? PAR : 0, A1 = (DA == 2) ? (PAR ^ 1) : 0;
        for (int s = 0; s < KB; s += 2) {
            if constexpr (LA) sync_read(NM{}, t0 + s, ra[0]);
            orbit_step<P, MASK>(xr[PAR], er[PAR], minus, ra[A0], acc);
            if constexpr (DA == 1 && !LA) load_a(min(t0 + s + 1, NIT - 1), ra[0]);
            load(NM{}, min(t0 + s + 2, NIT - 1), xr[PAR], ra[A0], er[PAR]);
            if constexpr (!LA) __builtin_amdgcn_sched_barrier(0);
            if (s + 1 < KB) {
                if constexpr (LA) sync_read(NM{}, t0 + s + 1, ra[0]);
                orbit_step<P, MASK>(xr[PAR ^ 1], er[PAR ^ 1], minus, ra[A1], acc);
                if constexpr (DA == 1 && !LA) load_a(min(t0 + s + 2, NIT - 1), ra[0]);
                load(NM{}, min(t0 + s + 3, NIT - 1), xr[PAR ^ 1], ra[A1], er[PAR ^ 1]);
                if constexpr (!LA) __builtin_amdgcn_sched_barrier(0);
            }
        }
    };
    auto orbit = [&](auto maskc, auto parc, int q) {
        // negative one-sign axes of the orbit (looked up with its member rows,
        // two steps before it starts)
        const int minus = mnext;
        run(maskc, parc, q, minus);
#pragma unroll
        for (int rb = 0; rb < NRB; ++rb) {
            // class sign (-1)^|c & minus| of the orbit's product
            const bool neg = __builtin_popcount(class_of_row_block(P, rb) & minus) & 1;
            const V4 pr = neg ? -acc[rb] : acc[rb];
            const V4 yk = pr - cmp[rb];
            const V4 tk = tot[rb] + yk;
            cmp[rb] = (tk - tot[rb]) - yk;
            tot[rb] = tk;
            acc[rb] = V4{0, 0, 0, 0};
        }
    };
    // the orbit groups in table order; with odd KB the first step of orbit q
    // uses slot q & 1
    auto group = [&](auto gic) {
        constexpr int GI = decltype(gic)::value;
        typedef std::integral_constant<int, kOrbGroupMask[GI]> MC;
        const int q0 = GI * kOrbGroup;
        if constexpr (KB & 1) {
            constexpr int P0 = (GI * kOrbGroup) & 1;
            for (int k = 0;; ++k) {
                orbit(MC{}, std::integral_constant<int, P0>{}, q0 + 2 * k);
                if (2 * k + 1 >= kOrbGroup) break;
                orbit(MC{}, std::integral_constant<int, P0 ^ 1>{}, q0 + 2 * k + 1);
            }
        } else {
            for (int k = 0; k < kOrbGroup; ++k) orbit(MC{}, std::integral_constant<int, 0>{}, q0 + k);
        }
    };
    static_assert(kOrbits == 8 * kOrbGroup, "eight orbit groups");
    group(std::integral_constant<int, 0>{});
    group(std::integral_constant<int, 1>{});
    group(std::integral_constant<int, 2>{});
    group(std::integral_constant<int, 3>{});
    group(std::integral_constant<int, 4>{});
    group(std::integral_constant<int, 5>{});
    group(std::integral_constant<int, 6>{});
    group(std::integral_constant<int, 7>{});
    // the last slab copies (of steps past the end) land before the wave ends
    if constexpr (LA) __builtin_amdgcn_s_waitcnt(waitcnt_vm_lgkm0(0));
    const int le = s_le[j];
    if (le < 0) return;
    // all row indices, then all current LE values, then the stores (loads in
    // flight together)
    int nat[NRB][4];
    float cur[NRB][4];
    float* lr = A.le + (size_t)le * KP;
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r) nat[rb][r] = A.orb_rows[16 * rb + 4 * g + r];
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r) cur[rb][r] = nat[rb][r] >= 0 ? lr[nat[rb][r]] : 0.0f;
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (nat[rb][r] >= 0) lr[nat[rb][r]] = cur[rb][r] + (tot[rb][r] - cmp[rb][r]);
}


// (tile schedule bit 3: operands gathered into registers instead of LDS)
template <int P>
void launch_m2l_orbit_p(const EvalArgs<float>& A, hipStream_t st)
{
    if ((A.tile_sched >> 3) & 1) hipLaunchKernelGGL((k_m2l_orbit<P, false>), dim3(A.n_tiles), dim3(256), 0, st, A);
    else hipLaunchKernelGGL((k_m2l_orbit<P, true>), dim3(A.n_tiles), dim3(256), 0, st, A);
}

}  // namespace lpb
