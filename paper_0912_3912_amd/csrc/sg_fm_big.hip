// sg_fm_big.hip -- the paper's pass-based local search with hill-climbing
// (Sec. IV, Fig. 3) on instances too large for a wavefront's LDS (more than
// 4096 spins): one wavefront per replica, the replica's state in device
// memory, and the unlocked spin of largest gain found through two levels of
// maxima.  The pass, its tie-break, best prefix, stopping rule and counters
// are those of the other pass kernels (sg_fm.hip).
//
// Per replica, in a slot of the scratch area (a wavefront takes replicas from
// a shared counter and reuses its slot):
//   half  int32 per spin (internal order): v_i = -s_i f_i, half the gain
//         -dE_i of moving i; kLocked once the spin has moved in the pass;
//   moves int32 per step of the pass: the internal index moved;
//   leaf  uint64 per group of 64 consecutive internal indices: the largest
//         key of its unlocked spins, key = (v + 2^31) << 32 | (2^32 - 1 - ext)
//         (larger gain first, then lower external index; 0: none unlocked);
// and in the wavefront's LDS the largest leaf key of every 64 leaves, whose
// wave-wide maximum is the move.  The key carries the mover's external index;
// int_of maps it to the internal one.  A move locks and flips the spin, adds
// its partners' half-gain changes (2 J s_i s_j for a coupling, 2 K s_i s_a s_b
// for a hyper-coupling) and recomputes the leaves it touched and their
// upper-level entries.  Spins stay in the replica's own row of the workspace.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "sg_launch.h"
#include "sg_layout.h"

namespace sg {

namespace {

constexpr int32_t kLocked = INT32_MIN;

template <int CTRL, int ROWS>
__device__ __forceinline__ uint64_t big_max_step(uint64_t v)
{
    const int lo = (int)(uint32_t)v, hi = (int)(uint32_t)(v >> 32);
    const uint32_t lo2 = (uint32_t)__builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWS, 0xF, false);
    const uint32_t hi2 = (uint32_t)__builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWS, 0xF, false);
    const uint64_t w = ((uint64_t)hi2 << 32) | lo2;
    return w > v ? w : v;
}

// Maximum over the 64 lanes (all active), as a wavefront-uniform value.
__device__ __forceinline__ uint64_t big_wave_max(uint64_t v)
{
    v = big_max_step<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
    v = big_max_step<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
    v = big_max_step<0x141, 0xF>(v);  // row_half_mirror
    v = big_max_step<0x140, 0xF>(v);  // row_mirror
    v = big_max_step<0x142, 0xA>(v);  // row_bcast:15
    v = big_max_step<0x143, 0xC>(v);  // row_bcast:31
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t big_key(int32_t v, uint32_t ext)
{
    if (v == kLocked) return 0ull;
    return ((uint64_t)((uint32_t)v ^ 0x80000000u) << 32) | (uint64_t)(0xFFFFFFFFu - ext);
}

// The wavefront's global stores are complete and visible to its later loads.
__device__ __forceinline__ void big_order()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

}  // namespace

// Grid: one 64-thread workgroup per slot.  Dynamic LDS: 8 * top_cap bytes of
// upper-level keys, then 4 * (c_cap + 1) bytes of colour row starts.
__global__ __launch_bounds__(64) void k_fm_big(const InstTab* __restrict__ tab, const int32_t* __restrict__ ctab,
                                               const uint32_t* const* __restrict__ int_of,
                                               const QueueItem* __restrict__ items, int nitems,
                                               uint32_t* __restrict__ counter, int32_t* __restrict__ half_all,
                                               int32_t* __restrict__ moves_all, uint64_t* __restrict__ leaf_all,
                                               int64_t slot_spins, int64_t slot_leaves, int top_cap,
                                               RepState* __restrict__ rs, CallStats* __restrict__ cs,
                                               uint32_t* __restrict__ err, int max_passes, int until_conv)
{
    extern __shared__ uint64_t big_lds[];
    uint64_t* top = big_lds;
    int32_t* crow = reinterpret_cast<int32_t*>(big_lds + top_cap);
    const int lane = threadIdx.x;
    int32_t* half = half_all + (int64_t)blockIdx.x * slot_spins;
    int32_t* moves = moves_all + (int64_t)blockIdx.x * slot_spins;
    uint64_t* leaf = leaf_all + (int64_t)blockIdx.x * slot_leaves;
    long long att = 0, kept_all = 0, passes_max = 0, unconv = 0;

    for (;;) {
        int k = 0;
        if (lane == 0) k = (int)atomicAdd(counter, 1u);
        k = __builtin_amdgcn_readfirstlane(k);
        if (k >= nitems) break;
        const QueueItem it = items[k];
        const InstTab& Q = tab[it.inst];
        const InstDev& I = Q.I;
        RepState* st = rs + Q.rep_base + it.r;
        if (st->converged) continue;
        const int n = I.n, G1 = (n + 63) >> 6, G2 = (G1 + 63) >> 6, C = Q.C;
        int8_t* sp = Q.spins + Q.spin_stride * it.r;
        const uint32_t* iof = int_of[it.inst];
        // first internal row of every colour (the slices of a colour are its
        // rows in chunks of 64 from that row)
        for (int c = lane; c <= C; c += 64) {
            const int s0 = ctab[Q.ctab_off + c];
            crow[c] = c < C ? (int)I.slices[s0].row0 : n;
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        long long Estar = st->E, kept = 0;
        int passes = 0;
        bool conv = false, bad = false;
        for (int pass = 0; pass < max_passes && !bad; ++pass) {
            // half-gains from the definition, slice by slice (lane = row)
            for (int sl = 0; sl < I.nslices; ++sl) {
                const Slice S = I.slices[sl];
                if (lane < S.rows) {
                    const int i = (int)S.row0 + lane;
                    int f = I.h[i];
                    const uint32_t* p = I.nbr + S.ebase + lane;
                    for (int q = 0; q < S.ew; ++q) {
                        const uint32_t w = p[q * kSlice];
                        f += (int)(int8_t)(w & 0xffu) * sp[w >> 8];
                    }
                    if (I.has_tri) {
                        const uint32_t* pa = I.ta + S.tbase + lane;
                        const uint32_t* pb = I.tb + S.tbase + lane;
                        for (int q = 0; q < S.tw; ++q) {
                            const uint32_t wa = pa[q * kSlice];
                            f += (int)(int8_t)(wa & 0xffu) * sp[wa >> 8] * sp[pb[q * kSlice]];
                        }
                    }
                    half[i] = -sp[i] * f;
                }
            }
            big_order();
            // leaves, then the upper level
            for (int g = 0; g < G1; ++g) {
                const int i = g * 64 + lane;
                const uint64_t key = i < n ? big_key(half[i], I.ext[i]) : 0ull;
                const uint64_t m = big_wave_max(key);
                if (lane == 0) leaf[g] = m;
            }
            big_order();
            for (int a = 0; a < G2; ++a) {
                const int g = a * 64 + lane;
                const uint64_t m = big_wave_max(g < G1 ? leaf[g] : 0ull);
                if (lane == 0) top[a] = m;
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            long long E = Estar, Elow = Estar;
            int best_len = 0;
            for (int step = 0; step < n; ++step) {
                // the move: the largest upper-level key
                uint64_t km = 0;
                for (int a = lane; a < G2; a += 64) km = top[a] > km ? top[a] : km;
                const uint64_t K = big_wave_max(km);
                const uint32_t ext = 0xFFFFFFFFu - (uint32_t)K;
                if (K == 0 || ext >= (uint32_t)n) {  // no unlocked spin before n moves: internal error
                    bad = true;
                    break;
                }
                const int v = (int)((uint32_t)(K >> 32) ^ 0x80000000u);
                const int i = (int)iof[ext];
                // its colour and slice
                const int cq = lane < C && crow[lane] <= i && i < crow[lane + 1] ? lane : -1;
                int c = -1;
                {
                    const uint64_t hit = __ballot(cq >= 0);
                    if (hit) c = __builtin_amdgcn_readlane(cq, __builtin_ctzll(hit));
                    for (int c0 = 64; c < 0 && c0 < C; c0 += 64)
                        for (int cc = c0; cc < min(C, c0 + 64) && c < 0; ++cc)
                            if (crow[cc] <= i && i < crow[cc + 1]) c = cc;
                }
                if (c < 0 || i < 0 || i >= n) {  // an index outside the instance: internal error
                    bad = true;
                    break;
                }
                const int rel = i - crow[c];
                const Slice S = I.slices[ctab[Q.ctab_off + c] + (rel >> 6)];
                const int l = rel & 63;
                const int s_old = sp[i];
                // partners: lane q takes coupling q and hyper-coupling q of the row
                int gj = -1, ga = -1, gb = -1;
                if (lane < S.ew) {
                    const uint32_t w = I.nbr[S.ebase + lane * kSlice + l];
                    const int J = (int)(int8_t)(w & 0xffu);
                    if (J) {
                        const int j = (int)(w >> 8);
                        const int32_t hv = half[j];
                        if (hv != kLocked) atomicAdd(&half[j], 2 * J * sp[j] * s_old);
                        gj = j >> 6;
                    }
                }
                if (I.has_tri && lane < S.tw) {
                    const uint32_t wa = I.ta[S.tbase + lane * kSlice + l];
                    const int K3 = (int)(int8_t)(wa & 0xffu);
                    if (K3) {
                        const int a = (int)(wa >> 8), b = (int)I.tb[S.tbase + lane * kSlice + l];
                        const int d = 2 * K3 * sp[a] * sp[b] * s_old;
                        if (half[a] != kLocked) atomicAdd(&half[a], d);
                        if (half[b] != kLocked) atomicAdd(&half[b], d);
                        ga = a >> 6;
                        gb = b >> 6;
                    }
                }
                if (lane == 0) {
                    half[i] = kLocked;
                    sp[i] = (int8_t)-s_old;
                    moves[step] = i;
                }
                E -= 2LL * v;
                if (E < Elow) {
                    Elow = E;
                    best_len = step + 1;
                }
                big_order();
                // the touched leaves (the mover's, then each distinct partner
                // leaf), up to four per round: their half-gains and the leaf
                // keys of their upper entries are read in one round trip, the
                // new leaf keys replace their old values in those entries, and
                // the entries' maxima are taken from registers
                int pend[3] = {gj, ga, gb};
                bool first = true;
                for (;;) {
                    int gl[4];
                    int ng = 0;
                    if (first) {
                        gl[ng++] = i >> 6;
                        first = false;
                    }
                    while (ng < 4) {
                        // the lowest pending leaf of any lane, cleared wherever it is pending
                        int cand = 0x7FFFFFFF;
                        for (int u = 0; u < 3; ++u)
                            if (pend[u] >= 0 && pend[u] < cand) cand = pend[u];
                        int g = cand;
                        for (int off = 32; off > 0; off >>= 1) g = min(g, __shfl_xor(g, off, 64));
                        if (g == 0x7FFFFFFF) break;
                        for (int u = 0; u < 3; ++u)
                            if (pend[u] == g) pend[u] = -1;
                        bool dup = false;
                        for (int u = 0; u < ng; ++u) dup = dup || gl[u] == g;
                        if (!dup) gl[ng++] = g;
                    }
                    if (ng == 0) break;
                    int32_t hv[4];
                    uint32_t ev[4];
                    uint64_t up[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int ii = u < ng ? gl[u] * 64 + lane : n;
                        hv[u] = ii < n ? half[ii] : kLocked;
                        ev[u] = ii < n ? I.ext[ii] : 0u;
                        const int gg = u < ng ? (gl[u] >> 6) * 64 + lane : G1;
                        up[u] = gg < G1 ? leaf[gg] : 0ull;
                    }
                    uint64_t kk[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) kk[u] = big_wave_max(big_key(hv[u], ev[u]));
                    // the new leaf keys into their entries' lanes, then each
                    // entry's maximum (an entry read twice gives the same value)
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        if (u >= ng) continue;
                        if (lane == 0) leaf[gl[u]] = kk[u];
#pragma unroll
                        for (int w = 0; w < 4; ++w)
                            if (w < ng && (gl[u] >> 6) == (gl[w] >> 6) && lane == (gl[u] & 63)) up[w] = kk[u];
                    }
#pragma unroll
                    for (int w = 0; w < 4; ++w) {
                        const uint64_t m = big_wave_max(up[w]);
                        if (w < ng && lane == 0) top[gl[w] >> 6] = m;
                    }
                    big_order();  // the leaf keys written before a later round reads them
                }
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            }
            if (bad) break;
            // undo the moves after the best prefix
            for (int t = best_len + lane; t < n; t += 64) {
                const int i = moves[t];
                sp[i] = (int8_t)-sp[i];
            }
            big_order();
            ++passes;
            kept += best_len;
            const bool improved = Elow < Estar;
            Estar = Elow;
            if (until_conv && !improved) {
                conv = true;
                break;
            }
        }
        if (bad) {
            if (lane == 0) atomicOr(err, 1u);
            continue;
        }
        if (lane == 0) {
            st->E = Estar;
            st->sweeps += passes;
            st->flips += kept;
            if (conv) st->converged = 1;
        }
        att += (long long)passes * n;
        kept_all += kept;
        passes_max = passes > passes_max ? passes : passes_max;
        unconv += (until_conv && !conv) ? 1 : 0;
    }
    if (lane == 0 && (att || unconv)) {
        atomicAdd(&cs->attempts, (unsigned long long)att);
        atomicAdd(&cs->flips, (unsigned long long)kept_all);
        atomicMax(&cs->sweeps_max, (unsigned long long)passes_max);
        atomicAdd(&cs->unconverged, (unsigned long long)unconv);
    }
}

size_t fm_big_lds_bytes(int top_cap, int c_cap) { return (size_t)top_cap * 8 + (size_t)(c_cap + 1) * 4; }

hipError_t launch_fm_big(const InstTab* tab, const int32_t* ctab, const uint32_t* const* int_of, const QueueItem* items,
                         int nitems, uint32_t* counter, int32_t* half, int32_t* moves, uint64_t* leaf,
                         int64_t slot_spins, int64_t slot_leaves, int slots, int top_cap, int c_cap, RepState* rs,
                         CallStats* cs, uint32_t* err, int max_passes, int until_conv, hipStream_t st)
{
    if (nitems <= 0 || slots <= 0) return hipSuccess;
    const size_t lds = fm_big_lds_bytes(top_cap, c_cap);
    hipError_t e = hipFuncSetAttribute((const void*)k_fm_big, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fm_big, dim3((unsigned)std::min(slots, nitems)), dim3(64), lds, st, tab, ctab, int_of, items,
                       nitems, counter, half, moves, leaf, slot_spins, slot_leaves, top_cap, rs, cs, err, max_passes,
                       until_conv);
    return hipGetLastError();
}

}  // namespace sg
