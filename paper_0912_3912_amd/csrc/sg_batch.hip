// sg_batch.hip -- the block schedule (one workgroup per instance and range of
// restarts) and the batched start and energy of many replicas.
//
// k_block: the instance's sliced couplings, its fields and the spins of RG
// (up to 256) restarts sit in LDS.  Spins are stored [spin][slot], so the 64
// lanes of a wavefront are 64 restarts of one spin: coupling reads are
// uniform across the wavefront (LDS broadcast) and spin reads are 64
// consecutive bytes.  A slot whose replica stops (converged, or its sweep
// budget spent) writes it back and takes the next restart of the range, so
// lanes do not idle while slower restarts of the same instance are still
// descending.  The replica state and the call totals follow the per-phase
// kernels exactly: with until_converged a replica stops after its first sweep
// without a flip (that sweep counts).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "sg_device.h"
#include "sg_launch.h"
#include "sg_layout.h"

namespace sg {

__device__ __forceinline__ int bat_j(uint32_t w) { return (int)(int8_t)(w & 0xffu); }

constexpr int kBatThreads = 1024;
constexpr int kBatWaves = kBatThreads / 64;

// ---------------------------------------------------------------------------
// k_block

template <bool TIE>
__global__ __launch_bounds__(kBatThreads) void k_block(const InstTab* __restrict__ tab, const int32_t* __restrict__ ctab,
                                                       const BlockItem* __restrict__ items, RepState* __restrict__ rs,
                                                       CallStats* __restrict__ cs, int RG, int T, uint64_t seed,
                                                       int until_conv)
{
    extern __shared__ uint64_t lds64[];
    const BlockItem it = items[blockIdx.x];
    const InstTab& Q = tab[it.inst];
    const InstDev& I = Q.I;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = I.n;
    const int r_end = it.r0 + it.nr;   // restarts [r0, r0 + nr) of the instance, RG at a time
    const int G = RG / 64;             // replica groups of 64 lanes
    const int S = kBatWaves / G;       // spin subsets
    const int g = wave % G, ss = wave / G;
    const int r_loc = g * 64 + lane;   // the lane's replica slot
    const bool owner = ss == 0;        // one thread per slot keeps its bookkeeping

    // LDS layout: couplings | triple words a | triple words b | slices | h | colour table | spins [n][RG] |
    // per-slot state
    const int ew = Q.nbr_words, tw = Q.tri_words, nsl = I.nslices, C = Q.C;
    uint32_t* l_nbr = reinterpret_cast<uint32_t*>(lds64);
    uint32_t* l_ta = l_nbr + ew;
    uint32_t* l_tb = l_ta + tw;
    Slice* l_sl = reinterpret_cast<Slice*>(l_tb + tw + ((ew + 2 * tw) & 3 ? 4 - ((ew + 2 * tw) & 3) : 0));
    int8_t* l_h = reinterpret_cast<int8_t*>(l_sl + nsl);
    int32_t* l_cs = reinterpret_cast<int32_t*>(l_h + ((n + 3) & ~3));
    int8_t* l_s = reinterpret_cast<int8_t*>(l_cs + C + 1);
    const size_t s_off = (size_t)(l_s - reinterpret_cast<int8_t*>(lds64));
    long long* sl_dE = reinterpret_cast<long long*>(reinterpret_cast<int8_t*>(lds64) +
                                                    ((s_off + (size_t)n * RG + 15) & ~(size_t)15));
    int* sl_r = reinterpret_cast<int*>(sl_dE + RG);  // restart in the slot, -1 when none
    int* sl_t = sl_r + RG;                           // its sweeps in this call
    uint32_t* sl_base = reinterpret_cast<uint32_t*>(sl_t + RG);  // its sweep index at the start of the call
    int* sl_last = reinterpret_cast<int*>(sl_base + RG);         // 1 + its last sweep that flipped
    int* sl_nf = sl_last + RG;                                   // its flips in this call
    int* sl_wb = sl_nf + RG;                                     // restart to write back from the slot, or -1
    int* sl_ld = sl_wb + RG;                                     // restart to load into the slot, or -1
    int* sw_flips = sl_ld + RG;                                  // flips of the current sweep
    __shared__ int n_live, next_r;
    __shared__ unsigned long long b_att, b_flips, b_smax, b_unconv;

    // coupling words staged with the partner's spin offset (j * RG, < 2^19)
    // in place of j: the lane's spin address is then one add
    for (int k = tid; k < ew; k += kBatThreads) {
        const uint32_t w = I.nbr[k];
        l_nbr[k] = (((w >> 8) * (uint32_t)RG) << 8) | (w & 0xffu);
    }
    if (I.has_tri)
        for (int k = tid; k < tw; k += kBatThreads) {
            const uint32_t wa = I.ta[k];
            l_ta[k] = (((wa >> 8) * (uint32_t)RG) << 8) | (wa & 0xffu);
            l_tb[k] = I.tb[k] * (uint32_t)RG;
        }
    for (int k = tid; k < nsl; k += kBatThreads) l_sl[k] = I.slices[k];
    for (int k = tid; k < n; k += kBatThreads) l_h[k] = I.h[k];
    for (int k = tid; k <= C; k += kBatThreads) l_cs[k] = ctab[Q.ctab_off + k];
    if (tid == 0) {
        n_live = 0;
        next_r = it.r0;
        b_att = b_flips = b_smax = b_unconv = 0;
    }
    if (tid < RG) sw_flips[tid] = 0;
    __syncthreads();

    // A replica leaves its slot: state and call totals (slot owner only).
    auto finalize = [&](int r, int t, int last, long long de, int nf) {
        RepState* st = rs + Q.rep_base + r;
        st->E += de;
        st->flips += nf;
        st->sweeps += t;
        st->lastflip = last;
        const bool conv = until_conv && last < t;
        if (conv) st->converged = 1;
        atomicAdd(&b_att, (unsigned long long)t * (unsigned long long)n);
        atomicAdd(&b_flips, (unsigned long long)nf);
        atomicMax(&b_smax, (unsigned long long)t);
        if (until_conv && !conv) atomicAdd(&b_unconv, 1ull);
    };
    // The next restart of the item that is not frozen (a replica that had
    // converged before the call keeps its state and is not counted), or -1.
    auto advance = [&]() -> int {
        for (;;) {
            const int rn = atomicAdd(&next_r, 1);
            if (rn >= r_end) return -1;
            const RepState s0 = rs[Q.rep_base + rn];
            if (s0.converged) continue;
            if (T <= 0) {
                finalize(rn, 0, 0, 0, 0);
                continue;
            }
            sl_t[r_loc] = 0;
            sl_base[r_loc] = (uint32_t)s0.sweeps;
            sl_last[r_loc] = 0;
            sl_dE[r_loc] = 0;
            sl_nf[r_loc] = 0;
            return rn;
        }
    };
    // Spins of the slot's outgoing and incoming replicas, rows of this subset.
    auto swap = [&]() {
        const int wb = sl_wb[r_loc], ld = sl_ld[r_loc];
        if (wb >= 0) {
            int8_t* gp = Q.spins + (int64_t)wb * Q.spin_stride;
            for (int i = ss; i < n; i += S) gp[i] = l_s[i * RG + r_loc];
        }
        if (ld >= 0) {
            const int8_t* gp = Q.spins + (int64_t)ld * Q.spin_stride;
            for (int i = ss; i < n; i += S) l_s[i * RG + r_loc] = gp[i];
        }
    };

    if (owner) {
        const int rn = advance();
        sl_r[r_loc] = rn;
        sl_wb[r_loc] = -1;
        sl_ld[r_loc] = rn;
        if (rn >= 0) atomicAdd(&n_live, 1);
    }
    __syncthreads();
    swap();
    __syncthreads();

    while (n_live > 0) {
        const int rr = sl_r[r_loc];
        const bool active = rr >= 0;
        const uint32_t r = active ? (uint32_t)rr : 0u;
        const uint32_t sweep = sl_base[r_loc] + (uint32_t)sl_t[r_loc];
        long long dE = 0;
        int my = 0;
        for (int c = 0; c < C; ++c) {
            const int s_lo = l_cs[c], s_hi = l_cs[c + 1];
            for (int sl = s_lo; sl < s_hi; ++sl) {
                const Slice Sl = l_sl[sl];
                for (int l = ss; l < Sl.rows; l += S) {
                    const int i = Sl.row0 + l;
                    int f = l_h[i];
                    const uint32_t* pw = l_nbr + Sl.ebase + l;
                    const int8_t* ls = l_s + r_loc;
                    // four couplings at a time: their loads are issued together
                    int kk = 0;
                    for (; kk + 4 <= Sl.ew; kk += 4) {
                        uint32_t w[4];
                        int sj[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) w[u] = pw[(kk + u) * kSlice];
#pragma unroll
                        for (int u = 0; u < 4; ++u) sj[u] = ls[w[u] >> 8];
#pragma unroll
                        for (int u = 0; u < 4; ++u) f += bat_j(w[u]) * sj[u];
                    }
                    for (; kk < Sl.ew; ++kk) {
                        const uint32_t w = pw[kk * kSlice];
                        f += bat_j(w) * ls[w >> 8];
                    }
                    if (I.has_tri) {
                        const uint32_t* pa = l_ta + Sl.tbase + l;
                        const uint32_t* pb = l_tb + Sl.tbase + l;
                        for (int kk2 = 0; kk2 < Sl.tw; ++kk2) {
                            const uint32_t wa = pa[kk2 * kSlice];
                            const uint32_t b = pb[kk2 * kSlice];
                            f += bat_j(wa) * ls[wa >> 8] * ls[b];
                        }
                    }
                    const int si = l_s[i * RG + r_loc];
                    const int d = 2 * si * f;
                    bool flip = d < 0;
                    if (TIE && d == 0 && active) flip = rng_bit(seed, I.ext[i], sweep, I.instance_id, r) != 0;
                    if (flip && active) {
                        l_s[i * RG + r_loc] = (int8_t)(-si);
                        dE += d;
                        ++my;
                    }
                }
            }
            __syncthreads();
        }
        // the sweep's totals per slot over the spin subsets
        if (my) {
            atomicAdd(&sw_flips[r_loc], my);
            atomicAdd(&sl_nf[r_loc], my);
        }
        if (dE) atomicAdd(reinterpret_cast<unsigned long long*>(&sl_dE[r_loc]), (unsigned long long)dE);
        __syncthreads();
        if (owner) {
            sl_wb[r_loc] = -1;
            sl_ld[r_loc] = -1;
            if (active) {
                const int t = ++sl_t[r_loc];
                const int tot = sw_flips[r_loc];
                sw_flips[r_loc] = 0;
                if (tot) sl_last[r_loc] = t;
                if ((until_conv && tot == 0) || t >= T) {
                    finalize(rr, t, sl_last[r_loc], sl_dE[r_loc], sl_nf[r_loc]);
                    const int rn = advance();
                    sl_r[r_loc] = rn;
                    sl_wb[r_loc] = rr;
                    sl_ld[r_loc] = rn;
                    if (rn < 0) atomicSub(&n_live, 1);
                }
            }
        }
        __syncthreads();
        swap();
        __syncthreads();
    }
    if (tid == 0) {
        if (b_att) atomicAdd(&cs->attempts, b_att);
        if (b_flips) atomicAdd(&cs->flips, b_flips);
        atomicMax(&cs->sweeps_max, b_smax);
        if (b_unconv) atomicAdd(&cs->unconverged, b_unconv);
    }
}

// ---------------------------------------------------------------------------
// batched start and energy: one block of 256 threads per replica listed in
// `reps` (handle replica indices); rep_inst maps a replica to its instance.

// Batched start of replicas cut into units of 1024 spins (any instance size,
// the grid spread over all units): draws the spins of the unit; the unit at
// spin 0 also resets the replica state (its energy is then set by k_energy_segs).
__global__ __launch_bounds__(256) void k_start_units(const InstTab* __restrict__ tab,
                                                     const StartUnit* __restrict__ units, RepState* __restrict__ rs,
                                                     uint64_t seed)
{
    const StartUnit u = units[blockIdx.x];
    const InstTab& Q = tab[u.inst];
    const uint32_t r = (uint32_t)(u.g - Q.rep_base);
    int8_t* sp = Q.spins + (int64_t)r * Q.spin_stride;
    const int end = min(Q.I.n, u.off + 1024);
    for (int i = u.off + threadIdx.x; i < end; i += blockDim.x)
        sp[i] = (int8_t)(rng_bit(seed, Q.I.ext[i], 0xFFFFFFFFu, Q.I.instance_id, r) ? -1 : 1);
    if (u.off == 0 && threadIdx.x == 0) {
        RepState z;
        z.E = 0; z.flips = 0; z.sweeps = 0; z.lastflip = 0; z.converged = 0;
        rs[u.g] = z;
    }
}

// Energy of replicas cut into units of four slices: each unit sums its rows'
// terms (each edge and triple at its smallest internal index) into part[unit];
// k_energy_segs then adds up the units of each replica.  (One atomic per unit
// on the replica's energy serialised thousands of units of a large instance.)
__global__ __launch_bounds__(256) void k_energy_units(const InstTab* __restrict__ tab,
                                                      const StartUnit* __restrict__ units, int64_t ubase,
                                                      int64_t* __restrict__ part_out)
{
    const StartUnit u = units[blockIdx.x];
    const InstTab& Q = tab[u.inst];
    const InstDev& I = Q.I;
    const int r = (int)(u.g - Q.rep_base);
    const int8_t* s = Q.spins + (int64_t)r * Q.spin_stride;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    long long acc = 0;
    const int sl = u.off + wave;
    if (sl < I.nslices) {
        const Slice S = I.slices[sl];
        if (lane < S.rows) {
            const int i = S.row0 + lane;
            const int si = s[i];
            int e = I.h[i] * si;
            const uint32_t* p = I.nbr + S.ebase + lane;
            // up to 16 coupling words, then their partners' spins, in flight together
            constexpr int kPre = 16;
            uint32_t w[kPre];
            int sj[kPre];
#pragma unroll
            for (int k = 0; k < kPre; ++k) w[k] = k < S.ew ? p[k * kSlice] : 0u;
#pragma unroll
            for (int k = 0; k < kPre; ++k) sj[k] = (k < S.ew && (int)(w[k] >> 8) > i) ? s[w[k] >> 8] : 0;
#pragma unroll
            for (int k = 0; k < kPre; ++k) e += bat_j(w[k]) * si * sj[k];
            for (int k = kPre; k < S.ew; ++k) {
                const uint32_t w1 = p[k * kSlice];
                const int j = (int)(w1 >> 8);
                if (j > i) e += bat_j(w1) * si * s[j];
            }
            if (I.has_tri) {
                const uint32_t* pa = I.ta + S.tbase + lane;
                const uint32_t* pb = I.tb + S.tbase + lane;
                for (int k = 0; k < S.tw; ++k) {
                    const uint32_t wa = pa[k * kSlice];
                    const int a = (int)(wa >> 8), b = (int)pb[k * kSlice];
                    if (a > i && b > i) e += bat_j(wa) * si * s[a] * s[b];
                }
            }
            acc = e;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    __shared__ long long wpart[4];
    if (lane == 0) wpart[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part_out[ubase + blockIdx.x] = -(wpart[0] + wpart[1] + wpart[2] + wpart[3]);
}

// Energy of each replica from its units' partial sums, one wavefront per
// replica: into rs[g].E, or into out[g] when out is given.
__global__ __launch_bounds__(256) void k_energy_segs(const EnergySeg* __restrict__ segs, int64_t nsegs,
                                                     const int64_t* __restrict__ part, RepState* __restrict__ rs,
                                                     int64_t* __restrict__ out)
{
    const int64_t k = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (k >= nsegs) return;
    const EnergySeg sg = segs[k];
    // eight independent loads in flight per lane (a 10^6-spin replica has ~4000 units)
    long long a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int64_t* pp = part + sg.u0;
    int u = lane;
    for (; u + 7 * 64 < sg.nu; u += 8 * 64) {
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] += pp[u + j * 64];
    }
    for (; u < sg.nu; u += 64) a[0] += pp[u];
    long long acc = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) {
        if (out) out[sg.g] = acc;
        else rs[sg.g].E = acc;
    }
}

hipError_t launch_start_units(const InstTab* tab, const StartUnit* start_units, int64_t n_start,
                              const StartUnit* energy_units, int64_t n_energy, const EnergySeg* segs, int64_t nsegs,
                              int64_t* part, RepState* rs, int64_t* out, uint64_t seed, bool init, hipStream_t st)
{
    if (init)
        for (int64_t b0 = 0; b0 < n_start; b0 += (1u << 30)) {
            const unsigned nb = (unsigned)std::min<int64_t>(n_start - b0, 1u << 30);
            hipLaunchKernelGGL(k_start_units, dim3(nb), dim3(256), 0, st, tab, start_units + b0, rs, seed);
        }
    for (int64_t b0 = 0; b0 < n_energy; b0 += (1u << 30)) {
        const unsigned nb = (unsigned)std::min<int64_t>(n_energy - b0, 1u << 30);
        hipLaunchKernelGGL(k_energy_units, dim3(nb), dim3(256), 0, st, tab, energy_units + b0, b0, part);
    }
    for (int64_t k0 = 0; k0 < nsegs; k0 += (int64_t)4 << 30) {
        const int64_t nk = std::min<int64_t>(nsegs - k0, (int64_t)4 << 30);
        hipLaunchKernelGGL(k_energy_segs, dim3((unsigned)((nk + 3) / 4)), dim3(256), 0, st, segs + k0, nk, part, rs,
                           out);
    }
    return hipGetLastError();
}

// Start and energy of many replicas of one instance, one lane per replica
// (items: instance, first restart, count <= 64; one wavefront per item).  A
// lane keeps its replica's spins bit-packed in its own LDS column (word w at
// bits[w * 64 + lane], bit set when s = -1, internal order), and the
// instance's slices and coupling words, the same for every lane, are walked
// in order with scalar loads.  INIT: draw the start (the Philox start rule)
// and store it as bytes; else read the stored spins.  Energy of Sec. II
// eq. (1) / Sec. VI eq. (5), each term at its smallest internal index.  An
// INIT item with a nonzero flag (BlockItem::pad) only draws its start and
// leaves E at 0: its energy comes later, from the kernel that runs its
// descent or from an energy pass before anything reads it.
template <bool INIT>
__global__ __launch_bounds__(256) void k_start_lanes(const InstTab* __restrict__ tab,
                                                     const BlockItem* __restrict__ items, int nitems, int wmax,
                                                     RepState* __restrict__ rs, int64_t* __restrict__ out,
                                                     uint64_t seed)
{
    extern __shared__ uint32_t lbits[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // wave-uniform item: its fields are read once into scalar registers (the
    // spin stores below could otherwise alias them and force reloads)
    const int item = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + wave);
    if (item >= nitems) return;
    const BlockItem it = items[item];
    const InstTab& Q = tab[it.inst];
    const int n = Q.I.n;
    // external indices through the constant address space: wave-uniform reads of
    // memory no kernel writes become scalar loads
    using cu32 = const __attribute__((address_space(4))) uint32_t;
    cu32* ext = (cu32*)Q.I.ext;
    const uint32_t iid = Q.I.instance_id;
    const int64_t stride = Q.spin_stride, rep_base = Q.rep_base;
    const uint32_t* __restrict__ ET = Q.eterm;
    const int n_eh = Q.n_eh, n_ee = Q.n_ee, n_et = Q.n_et;
    const int W = (n + 31) >> 5;
    uint32_t* bits = lbits + (size_t)wave * wmax * 64;
    const bool mine = lane < it.nr;
    const int r = it.r0 + (mine ? lane : 0);
    int8_t* sp = Q.spins + stride * r;
    if (!INIT) {
        // stored spins: 32 bytes per word in two 16-byte loads (a replica's
        // spin row is padded past n to a multiple of 256 bytes); the sign bits
        // of four bytes gather by one multiply (no carries reach bits 28-31)
        auto signs4 = [](uint32_t x) -> uint32_t { return ((x & 0x80808080u) * 0x00204081u) >> 28; };
        for (int w = 0; w < W; ++w) {
            const uint4 a = *reinterpret_cast<const uint4*>(sp + w * 32);
            const uint4 b = *reinterpret_cast<const uint4*>(sp + w * 32 + 16);
            uint32_t word = signs4(a.x) | (signs4(a.y) << 4) | (signs4(a.z) << 8) | (signs4(a.w) << 12) |
                            (signs4(b.x) << 16) | (signs4(b.y) << 20) | (signs4(b.z) << 24) | (signs4(b.w) << 28);
            const int left = n - w * 32;
            if (left < 32) word &= (1u << left) - 1u;
            bits[w * 64 + lane] = word;
        }
    }
    // a drawn start: spins by the start rule, 32 bytes per word in two 16-byte
    // stores (bytes past n, inside the row's padding, hold +1)
    for (int w = 0; INIT && w < W; ++w) {
        uint32_t word = 0;
        uint32_t qv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int i0 = w * 32 + 4 * q;
            uint32_t quad = 0x01010101u;
            if (i0 + 4 <= n) {
                // four counters read together, then four independent draws
                uint32_t e[4];
#pragma unroll
                for (int b = 0; b < 4; ++b) e[b] = ext[i0 + b];
                quad = 0;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int neg = rng_bit(seed, e[b], 0xFFFFFFFFu, iid, (uint32_t)r);
                    word |= (uint32_t)neg << (4 * q + b);
                    quad |= (neg ? 0xFFu : 0x01u) << (8 * b);
                }
            } else if (i0 < n) {
                for (int b = 0; i0 + b < n; ++b) {
                    const int neg = rng_bit(seed, ext[i0 + b], 0xFFFFFFFFu, iid, (uint32_t)r);
                    word |= (uint32_t)neg << (4 * q + b);
                    if (neg) quad ^= 0xFEu << (8 * b);
                }
            }
            qv[q] = quad;
        }
        if (mine) {
            uint4* dst = reinterpret_cast<uint4*>(sp + w * 32);
            dst[0] = make_uint4(qv[0], qv[1], qv[2], qv[3]);
            dst[1] = make_uint4(qv[4], qv[5], qv[6], qv[7]);
        }
        bits[w * 64 + lane] = word;
    }
    if (INIT && it.pad) {
        if (mine) {
            RepState z;
            z.E = 0; z.flips = 0; z.sweeps = 0; z.lastflip = 0; z.converged = 0;
            rs[rep_base + r] = z;
        }
        return;
    }
    // -E as a sum over the instance's term list (the same for every lane):
    // a product of spins is +1 or -1 by the parity of their set bits
    auto bit = [&](uint32_t j) -> uint32_t { return (bits[(j >> 5) * 64 + lane] >> (j & 31u)) & 1u; };
    auto coef = [](uint32_t w) -> int { return (int)(int8_t)(uint8_t)(w >> 22); };
    int e2 = 0;  // |sum| < 2048 * 128 + 2048^2 / 2 * 128 < 2^31
    const uint32_t* et = ET;
#pragma unroll 8
    for (int t = 0; t < n_eh; ++t) {
        const uint32_t w = et[t];
        e2 += bit(w & 0x7FFu) ? -coef(w) : coef(w);
    }
    et += n_eh;
#pragma unroll 8
    for (int t = 0; t < n_ee; ++t) {
        const uint32_t w = et[t];
        e2 += (bit(w & 0x7FFu) ^ bit((w >> 11) & 0x7FFu)) ? -coef(w) : coef(w);
    }
    et += n_ee;
    long long acc = e2;
#pragma unroll 4
    for (int t = 0; t < n_et; ++t) {
        const uint32_t w = et[2 * t], b = et[2 * t + 1];
        acc += (bit(w & 0x7FFu) ^ bit((w >> 11) & 0x7FFu) ^ bit(b)) ? -coef(w) : coef(w);
    }
    if (mine) {
        const int64_t g = rep_base + r;
        if (INIT) {
            RepState z;
            z.E = -acc; z.flips = 0; z.sweeps = 0; z.lastflip = 0; z.converged = 0;
            rs[g] = z;
        } else if (out) {
            out[g] = -acc;
        } else {
            rs[g].E = -acc;
        }
    }
}

hipError_t launch_start_lanes(const InstTab* tab, const BlockItem* items, int nitems, int nmax, bool init,
                              RepState* rs, int64_t* out, uint64_t seed, hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    const int wmax = (nmax + 31) / 32;
    const size_t lds = (size_t)4 * wmax * 64 * 4;
    if (lds > 65536) return hipErrorInvalidValue;
    const dim3 grid((nitems + 3) / 4);
    if (init)
        hipLaunchKernelGGL(k_start_lanes<true>, grid, dim3(256), lds, st, tab, items, nitems, wmax, rs, out, seed);
    else
        hipLaunchKernelGGL(k_start_lanes<false>, grid, dim3(256), lds, st, tab, items, nitems, wmax, rs, out, seed);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// launchers

size_t block_lds_bytes(int n, int nbr_words, int tri_words, int nslices, int C, int RG)
{
    size_t b = (size_t)nbr_words * 4 + (size_t)tri_words * 8;
    b = (b + 15) / 16 * 16;
    b += (size_t)nslices * sizeof(Slice);
    b += (size_t)((n + 3) & ~3);
    b += (size_t)(C + 1) * 4;
    b += (size_t)n * RG;
    b = (b + 15) / 16 * 16;
    b += (size_t)RG * 40;  // per-slot state
    return (b + 15) / 16 * 16;
}

hipError_t launch_block(const InstTab* tab, const int32_t* ctab, const BlockItem* items, int n_items, size_t lds,
                        RepState* rs, CallStats* cs, int RG, int T, uint64_t seed, int rule, int until_conv,
                        hipStream_t st)
{
    const void* kern = rule == 1 ? (const void*)k_block<true> : (const void*)k_block<false>;
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (rule == 1)
        hipLaunchKernelGGL(k_block<true>, dim3(n_items), dim3(kBatThreads), lds, st, tab, ctab, items, rs, cs, RG, T,
                           seed, until_conv);
    else
        hipLaunchKernelGGL(k_block<false>, dim3(n_items), dim3(kBatThreads), lds, st, tab, ctab, items, rs, cs, RG, T,
                           seed, until_conv);
    return hipGetLastError();
}

int block_max_blocks(size_t lds)
{
    const void* kern = (const void*)k_block<true>;
    int per_cu = 0, dev = 0, cus = 0;
    if (hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kBatThreads, lds) != hipSuccess ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return per_cu * cus;
}

}  // namespace sg
