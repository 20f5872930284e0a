// sg_fm_big.hip -- the paper's pass-based local search with hill-climbing
// (Sec. IV, Fig. 3) on instances too large for a wavefront's LDS (more than
// 4096 spins): one wavefront per replica, the replica's state in device
// memory, and the unlocked spin of largest gain found through two levels of
// maxima.  The pass, its tie-break, best prefix, stopping rule and counters
// are those of the other pass kernels (sg_fm.hip).
//
// Everything here is in external order, so that the largest key names its
// spin directly.  Per instance a row table (FmbRows): per spin a word with
// its field, then dc couplings and tt hyper-couplings, unused entries zero:
// in the packed form words partner << 8 | J & 255 and pairs (a << 8 | K &
// 255, b), in the wide form (any int32 coefficient) pairs (partner, J) and
// triples (a, b, K).  A move's terms are taken 64 at a time (a lane each).  Per
// replica, in a slot of the scratch area (a wavefront takes replicas from a
// shared counter and reuses its slot):
//   half  int32 per spin: v_e = -s_e f_e, half the gain -dE_e of moving e;
//         kLocked once the spin has moved in the pass;
//   spin  int8 per spin (copied from and back to the replica's own row, which
//         is in internal order);
//   moves int32 per step of the pass: the spin moved;
//   leaf  uint64 per group of 64 consecutive spins: the largest key of its
//         unlocked spins, key = (v + 2^31) << 32 | (2^32 - 1 - e) (larger gain
//         first, then lower index; 0: none unlocked);
// and in the wavefront's LDS the largest leaf key of every 64 leaves, whose
// wave-wide maximum is the move.  A move locks and flips the spin, adds its
// partners' half-gain changes (2 J s_e s_j for a coupling, 2 K s_e s_a s_b
// for a hyper-coupling) and recomputes the leaves it touched and their
// upper-level entries: the touched leaves are gathered whole, the changes
// added in LDS and the results stored, so that a move costs two dependent
// device-memory round trips (its row, then the gather) when it touches at
// most four leaves.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "sg_launch.h"
#include "sg_layout.h"

namespace sg {

namespace {

constexpr int32_t kLocked = INT32_MIN;

// The row table as device memory (its pointer comes from a table in memory,
// so the compiler would otherwise address it as generic memory).
typedef __attribute__((address_space(1))) const uint32_t fmb_g32;

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

__device__ __forceinline__ uint64_t big_key(int32_t v, uint32_t e)
{
    if (v == kLocked) return 0ull;
    return ((uint64_t)((uint32_t)v ^ 0x80000000u) << 32) | (uint64_t)(0xFFFFFFFFu - e);
}

// The wavefront's device-memory stores and atomics are complete and visible
// to its later loads.
__device__ __forceinline__ void big_order()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

}  // namespace

// Grid: one 64-thread workgroup per slot.  Dynamic LDS: 8 * top_cap bytes.
__global__ __launch_bounds__(64) void k_fm_big(const InstTab* __restrict__ tab, const FmbRows* __restrict__ rows,
                                               const QueueItem* __restrict__ items, int nitems,
                                               uint32_t* __restrict__ counter, int32_t* __restrict__ half_all,
                                               int32_t* __restrict__ moves_all, uint64_t* __restrict__ leaf_all,
                                               int8_t* __restrict__ spin_all, int64_t slot_spins, int64_t slot_leaves,
                                               RepState* __restrict__ rs, CallStats* __restrict__ cs,
                                               uint32_t* __restrict__ err, int max_passes, int until_conv)
{
    extern __shared__ uint64_t top[];
    __shared__ int32_t dl[4 * 64];  // a round's half-gain changes per gathered leaf and lane
    const int lane = threadIdx.x;
    for (int u = 0; u < 4; ++u) dl[u * 64 + lane] = 0;
    int32_t* half = half_all + (int64_t)blockIdx.x * slot_spins;
    int32_t* moves = moves_all + (int64_t)blockIdx.x * slot_spins;
    int8_t* sx = spin_all + (int64_t)blockIdx.x * slot_spins;
    uint64_t* leaf = leaf_all + (int64_t)blockIdx.x * slot_leaves;
    long long att = 0, kept_all = 0, passes_max = 0, unconv = 0;

    for (;;) {
        int k = 0;
        if (lane == 0) k = (int)atomicAdd(counter, 1u);
        k = __builtin_amdgcn_readfirstlane(k);
        if (k >= nitems) break;
        const QueueItem it = items[k];
        const InstTab& Q = tab[it.inst];
        const FmbRows Rw = rows[it.inst];
        RepState* st = rs + Q.rep_base + it.r;
        if (st->converged) continue;
        const int n = Q.I.n, G1 = (n + 63) >> 6, G2 = (G1 + 63) >> 6;
        const int dc = Rw.dc, tt = Rw.tt, stride = Rw.stride;
        int8_t* sp = Q.spins + Q.spin_stride * it.r;
        const uint32_t* ext = Q.I.ext;
        // the replica's spins into external order
        for (int i = lane; i < n; i += 64) sx[ext[i]] = sp[i];
        big_order();
        long long Estar = st->E, kept = 0;
        int passes = 0;
        bool conv = false, bad = false;
        for (int pass = 0; pass < max_passes && !bad; ++pass) {
            // half-gains from the definition, 64 spins at a time (every
            // partial sum of a field is bounded by the spin's sum of |c|,
            // below 2^31)
            for (int e = lane; e < n; e += 64) {
                fmb_g32* row = (fmb_g32*)Rw.rows + (int64_t)e * stride;
                int f;
                if (!Rw.wide) {
                    f = (int)(int8_t)(row[0] & 0xffu);
                    for (int q = 0; q < dc; ++q) {
                        const uint32_t w = row[1 + q];
                        f += (int)(int8_t)(w & 0xffu) * sx[w >> 8];
                    }
                    for (int q = 0; q < tt; ++q) {
                        const uint32_t wa = row[1 + dc + 2 * q], b = row[2 + dc + 2 * q];
                        f += (int)(int8_t)(wa & 0xffu) * sx[wa >> 8] * sx[b];
                    }
                } else {
                    f = (int)row[0];
                    for (int q = 0; q < dc; ++q) f += (int)row[2 + 2 * q] * sx[row[1 + 2 * q]];
                    for (int q = 0; q < tt; ++q) {
                        fmb_g32* t3 = row + 1 + 2 * dc + 3 * q;
                        f += (int)t3[2] * sx[t3[0]] * sx[t3[1]];
                    }
                }
                half[e] = -sx[e] * f;
            }
            big_order();
            // leaves, then the upper level
            for (int g = 0; g < G1; ++g) {
                const int e = g * 64 + lane;
                const uint64_t m = big_wave_max(e < n ? big_key(half[e], (uint32_t)e) : 0ull);
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
                const uint32_t me = 0xFFFFFFFFu - (uint32_t)K;
                if (K == 0 || me >= (uint32_t)n) {  // no unlocked spin before n moves: internal error
                    bad = true;
                    break;
                }
                const int v = (int)((uint32_t)(K >> 32) ^ 0x80000000u);
                fmb_g32* row = (fmb_g32*)Rw.rows + (int64_t)me * stride;
                const int s_old = sx[me];
                const int gm = (int)(me >> 6);
                E -= 2LL * v;
                if (E < Elow) {
                    Elow = E;
                    best_len = step + 1;
                }
                // the mover's terms, 64 at a time (lane: coupling q and
                // hyper-coupling q); a partner's half-gain changes by
                // 2 J s_j s_old or 2 K s_a s_b s_old, added modulo 2^32 (every
                // value it ends at is in range)
                const int nq = dc > tt ? dc : tt;
                for (int q0 = 0; q0 == 0 || q0 < nq; q0 += 64) {
                    const int q = q0 + lane;
                    int j = 0, a = 0, b = 0;
                    int32_t J = 0, K3 = 0;
                    if (!Rw.wide) {
                        const uint32_t w = q < dc ? row[1 + q] : 0u;
                        const uint32_t wa = q < tt ? row[1 + dc + 2 * q] : 0u;
                        j = (int)(w >> 8);
                        J = (int)(int8_t)(w & 0xffu);
                        a = (int)(wa >> 8);
                        b = q < tt ? (int)row[2 + dc + 2 * q] : 0;
                        K3 = (int)(int8_t)(wa & 0xffu);
                    } else {
                        if (q < dc) {
                            j = (int)row[1 + 2 * q];
                            J = (int32_t)row[2 + 2 * q];
                        }
                        if (q < tt) {
                            fmb_g32* t3 = row + 1 + 2 * dc + 3 * q;
                            a = (int)t3[0];
                            b = (int)t3[1];
                            K3 = (int32_t)t3[2];
                        }
                    }
                    // the touched leaves (the mover's, then each distinct
                    // partner leaf), up to four per round.  A round gathers
                    // their half-gains and the leaf keys of their upper
                    // entries in one round trip (the first round also the
                    // partners' spins), adds the partners it takes through
                    // the LDS table dl, stores the changed half-gains and
                    // leaf keys and refreshes the upper entries from
                    // registers.
                    int pend[3] = {J ? j >> 6 : -1, K3 ? a >> 6 : -1, K3 ? b >> 6 : -1};
                    bool first = q0 == 0, fresh = true;
                    int32_t dJ = 0, dK = 0;
                    for (;;) {
                        int gl[4];
                        int ng = 0;
                        bool take[3] = {false, false, false};
                        if (first) {
                            gl[ng++] = gm;
                            first = false;
                        }
                        while (ng < 4) {
                            // the pending leaf of the first lane that has one,
                            // taken wherever it is pending
                            const uint64_t b0 = __ballot(pend[0] >= 0), b1 = __ballot(pend[1] >= 0),
                                           b2 = __ballot(pend[2] >= 0);
                            int g;
                            if (b0)
                                g = __builtin_amdgcn_readlane(pend[0], (int)__builtin_ctzll(b0));
                            else if (b1)
                                g = __builtin_amdgcn_readlane(pend[1], (int)__builtin_ctzll(b1));
                            else if (b2)
                                g = __builtin_amdgcn_readlane(pend[2], (int)__builtin_ctzll(b2));
                            else
                                break;
                            for (int u = 0; u < 3; ++u)
                                if (pend[u] == g) {
                                    pend[u] = -1;
                                    take[u] = true;
                                }
                            bool dup = false;
                            for (int u = 0; u < ng; ++u) dup = dup || gl[u] == g;
                            if (!dup) gl[ng++] = g;
                        }
                        if (ng == 0) break;
                        // earlier stores (the previous move's, an earlier
                        // round's) are complete before the gather reads them
                        big_order();
                        if (fresh) {
                            const int sj = J ? sx[j] : 0, sa = K3 ? sx[a] : 0, sb = K3 ? sx[b] : 0;
                            dJ = (int32_t)((uint32_t)J * (uint32_t)(2 * sj * s_old));
                            dK = (int32_t)((uint32_t)K3 * (uint32_t)(2 * sa * sb * s_old));
                            fresh = false;
                        }
                        int32_t hv[4];
                        uint32_t ev[4];
                        uint64_t up[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int e = u < ng ? gl[u] * 64 + lane : n;
                            ev[u] = (uint32_t)e;
                            hv[u] = e < n ? half[e] : kLocked;
                            const int gg = u < ng ? (gl[u] >> 6) * 64 + lane : G1;
                            up[u] = gg < G1 ? leaf[gg] : 0ull;
                        }
                        // this round's partners into their leaves' rows of dl
                        // (same-wavefront LDS operations complete in order)
                        const int pe[3] = {j, a, b};
                        const int32_t pd[3] = {dJ, dK, dK};
#pragma unroll
                        for (int u = 0; u < 3; ++u) {
                            if (!take[u]) continue;
                            int x = 0;
                            for (int y = 1; y < ng; ++y)
                                if (gl[y] == (pe[u] >> 6)) x = y;
                            atomicAdd(&dl[x * 64 + (pe[u] & 63)], pd[u]);
                        }
                        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                        uint64_t kk[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            int32_t nv = hv[u];
                            if (u < ng) {
                                const int32_t add = dl[u * 64 + lane];
                                dl[u * 64 + lane] = 0;
                                if (nv != kLocked) nv = (int32_t)((uint32_t)nv + (uint32_t)add);
                                if (ev[u] == me) nv = kLocked;
                                if (nv != hv[u]) half[ev[u]] = nv;
                            }
                            kk[u] = big_wave_max(big_key(nv, ev[u]));
                        }
                        // the old keys of the gathered leaves (lane gl & 63 of their
                        // entries' keys), then the new keys into those lanes
                        uint64_t oldk[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int src = u < ng ? (gl[u] & 63) : 0;
                            const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)up[u], src);
                            const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(up[u] >> 32), src);
                            oldk[u] = ((uint64_t)hi << 32) | lo;
                        }
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            if (u >= ng) continue;
                            if (lane == 0) leaf[gl[u]] = kk[u];
#pragma unroll
                            for (int x = 0; x < 4; ++x)
                                if (x < ng && (gl[u] >> 6) == (gl[x] >> 6) && lane == (gl[u] & 63)) up[x] = kk[u];
                        }
                        // each touched entry once: its new maximum is the larger of
                        // its old one and the new keys, unless a leaf that held the
                        // old maximum went down (keys are distinct but for 0, below
                        // which none goes); then its 64 leaf keys are taken again
#pragma unroll
                        for (int x = 0; x < 4; ++x) {
                            if (x >= ng) continue;
                            const int a = gl[x] >> 6;
                            bool again = false;
                            for (int y = 0; y < x; ++y) again = again || (gl[y] >> 6) == a;
                            if (again) continue;
                            const uint64_t t0 = top[a];
                            const uint64_t told =
                                ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(t0 >> 32)) << 32) |
                                (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)t0);
                            uint64_t m = told;
                            bool down = false;
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
                                if (u >= ng || (gl[u] >> 6) != a) continue;
                                down = down || (oldk[u] == told && kk[u] < oldk[u]);
                                m = kk[u] > m ? kk[u] : m;
                            }
                            if (down) m = big_wave_max(up[x]);
                            if (lane == 0) top[a] = m;
                        }
                        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    }
                }
                if (lane == 0) {
                    sx[me] = (int8_t)-s_old;
                    moves[step] = (int)me;
                }
            }
            big_order();  // the last moves' stores before the undo reads them
            if (bad) break;
            // undo the moves after the best prefix
            for (int t = best_len + lane; t < n; t += 64) {
                const int e = moves[t];
                sx[e] = (int8_t)-sx[e];
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
        // the spins back into the replica's row (internal order)
        for (int i = lane; i < n; i += 64) sp[i] = sx[ext[i]];
        if (lane == 0) {
            st->E = Estar;
            st->sweeps += passes;
            st->flips += kept;
            if (conv) st->converged = 1;
        }
        big_order();
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

hipError_t launch_fm_big(const InstTab* tab, const FmbRows* rows, const QueueItem* items, int nitems,
                         uint32_t* counter, int32_t* half, int32_t* moves, uint64_t* leaf, int8_t* spins,
                         int64_t slot_spins, int64_t slot_leaves, int slots, int top_cap, RepState* rs, CallStats* cs,
                         uint32_t* err, int max_passes, int until_conv, hipStream_t st)
{
    if (nitems <= 0 || slots <= 0) return hipSuccess;
    const size_t lds = (size_t)top_cap * 8;
    hipError_t e = hipFuncSetAttribute((const void*)k_fm_big, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fm_big, dim3((unsigned)std::min(slots, nitems)), dim3(64), lds, st, tab, rows, items, nitems,
                       counter, half, moves, leaf, spins, slot_spins, slot_leaves, rs, cs, err, max_passes,
                       until_conv);
    return hipGetLastError();
}

}  // namespace sg
