// sg_queue.hip -- the persistent queue schedule for many instances of uneven
// size: workgroups take (instance, restart) items from a queue sorted by
// decreasing size.  Large items run on the whole workgroup (rows of the
// sliced layout on lanes, couplings streamed from memory, spins in LDS);
// small items run one per wavefront in a private LDS window, 16 at a time.
// Each replica runs to its own stopping point, and the replica state and the
// call totals follow the per-phase kernels exactly: with until_converged a
// replica stops after its first sweep without a flip (that sweep counts).
// A sweep without a flip evaluates every spin on the final configuration, so
// its fields also give the replica's exact energy, which is then stored
// instead of the running sum (the start energy is not needed for it).
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
// k_queue

// One colour phase of one replica on `nw` wavefronts (wave index w among
// them): lane = row of a slice, couplings from memory, spins in LDS.  All
// coupling and hyper-coupling words of a slice (up to kPreW and kPreT of
// them, predicated on the slice's widths) are loaded before any is used, so a
// wavefront keeps a whole slice's loads in flight (measured on 2000 uneven
// instances: 3.26 ms, against 4.67 ms with four loads at a time and 3.78 ms
// when loading the next slice while evaluating the current one with fewer
// words each).  The slice descriptors are read with scalar loads one slice
// ahead and the instance arrays addressed as device memory (2.78 ms; with
// the descriptor read per lane before the words and generic loads, 3.25 ms;
// 2.70 ms once a workgroup item's next-phase first slices are loaded before
// the phase barrier, queue_phase_wg).
// Loading the next slice's words as well, with both buffers at full width,
// measured 2.82-2.89 ms: the extra registers and copies cost more than the
// latency they hide.
constexpr int kPreW = 16, kPreT = 8;

struct SliceWords {
    uint32_t w[kPreW];
    uint32_t a[kPreT], b[kPreT];
    int h;
};

// Device-memory views of the instance arrays (the pointers come from the
// instance table, so the compiler would otherwise address them as generic
// memory, whose loads also hold up every LDS wait), and a read-only view of
// the slice table for loads at wavefront-uniform addresses (scalar loads).
typedef __attribute__((address_space(1))) const uint32_t q_g32;
typedef __attribute__((address_space(1))) const int8_t q_gi8;
typedef uint32_t q_v4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(4))) const q_v4 q_kslice;

__device__ __forceinline__ q_v4 queue_slice_raw(const Slice* slices, int sl) { return *(q_kslice*)(slices + sl); }

__device__ __forceinline__ Slice queue_unpack(q_v4 v)
{
    Slice S;
    S.row0 = v.x;
    S.ebase = v.y;
    S.tbase = v.z;
    S.ew = (uint16_t)(v.w & 0xFFFFu);
    S.tw = (uint8_t)((v.w >> 16) & 0xFFu);
    S.rows = (uint8_t)(v.w >> 24);
    return S;
}

// A pointer the whole wavefront holds, in scalar registers.
template <class T>
__device__ __forceinline__ T* queue_uniform(T* p)
{
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return (T*)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ void queue_load(const InstDev& I, const Slice& S, int lane, SliceWords& L)
{
    const bool row = lane < S.rows;
    q_g32* p = (q_g32*)I.nbr + S.ebase + lane;
#pragma unroll
    for (int k = 0; k < kPreW; ++k) L.w[k] = (row && k < S.ew) ? p[k * kSlice] : 0u;
    if (I.has_tri) {
        q_g32* pa = (q_g32*)I.ta + S.tbase + lane;
        q_g32* pb = (q_g32*)I.tb + S.tbase + lane;
#pragma unroll
        for (int q = 0; q < kPreT; ++q) {
            L.a[q] = (row && q < S.tw) ? pa[q * kSlice] : 0u;
            L.b[q] = (row && q < S.tw) ? pb[q * kSlice] : 0u;
        }
    }
    L.h = row ? (int)((q_gi8*)I.h)[S.row0 + lane] : 0;
}

// Energy from one sweep's fields: with f1 = h_i + (coupling part) and f the
// whole field, sum_i s_i (3 h_i + f1_i + 2 f_i) = 6 (sum h s + sum_{i<j} J s s
// + sum K s s s) = -6 E, each pair counted twice and each triple three times
// in the fields (Sec. II eq. (1), Sec. VI eq. (5)).
template <bool TIE>
__device__ __forceinline__ void queue_eval(const InstDev& I, const Slice& S, const SliceWords& L,
                                           int8_t* __restrict__ sp, int lane, uint32_t sweep, uint64_t seed,
                                           uint32_t r, long long& dE, int& my, long long& e6)
{
    if (lane >= S.rows) return;
    const int i = S.row0 + lane;
    int f = L.h;
#pragma unroll
    for (int k = 0; k < kPreW; ++k)
        if (k < S.ew) f += bat_j(L.w[k]) * sp[L.w[k] >> 8];
    if (S.ew > kPreW) {
        q_g32* p = (q_g32*)I.nbr + S.ebase + lane;
        for (int k = kPreW; k < S.ew; ++k) {
            const uint32_t w1 = p[k * kSlice];
            f += bat_j(w1) * sp[w1 >> 8];
        }
    }
    const int f1 = f;
    if (I.has_tri) {
#pragma unroll
        for (int q = 0; q < kPreT; ++q)
            if (q < S.tw) f += bat_j(L.a[q]) * sp[L.a[q] >> 8] * sp[L.b[q]];
        if (S.tw > kPreT) {
            q_g32* pa = (q_g32*)I.ta + S.tbase + lane;
            q_g32* pb = (q_g32*)I.tb + S.tbase + lane;
            for (int q = kPreT; q < S.tw; ++q) {
                const uint32_t wa = pa[q * kSlice];
                f += bat_j(wa) * sp[wa >> 8] * sp[pb[q * kSlice]];
            }
        }
    }
    const int si = sp[i];
    e6 += si * (3 * L.h + f1 + 2 * f);
    const int d = 2 * si * f;
    bool flip = d < 0;
    if (TIE && d == 0) flip = rng_bit(seed, ((q_g32*)I.ext)[i], sweep, I.instance_id, r) != 0;
    if (flip) {
        sp[i] = (int8_t)(-si);
        dE += d;
        ++my;
    }
}

template <bool TIE>
__device__ __forceinline__ void queue_phase(const InstDev& I0, const Slice* __restrict__ slices0, int s_lo, int s_hi,
                                            int8_t* __restrict__ sp, int w, int nw, int lane, uint32_t sweep,
                                            uint64_t seed, uint32_t r, long long& dE, int& my, long long& e6)
{
    InstDev I = I0;
    I.nbr = queue_uniform(I0.nbr);
    I.ta = queue_uniform(I0.ta);
    I.tb = queue_uniform(I0.tb);
    I.h = queue_uniform(I0.h);
    I.ext = queue_uniform(I0.ext);
    const Slice* slices = queue_uniform(slices0);
    // the next slice's descriptor is read while this slice's words are in
    // flight, so a slice costs one memory latency, not two
    int sl = __builtin_amdgcn_readfirstlane(s_lo + w);
    q_v4 nx = {0u, 0u, 0u, 0u};
    if (sl < s_hi) nx = queue_slice_raw(slices, sl);
    for (; sl < s_hi; sl += nw) {
        // the descriptor is first used here, one slice after its load was
        // issued (the empty statement keeps the compiler from unpacking, and
        // so waiting for, it right after the load)
        asm volatile("" : "+s"(nx.x), "+s"(nx.y), "+s"(nx.z), "+s"(nx.w));
        const Slice S = queue_unpack(nx);
        if (sl + nw < s_hi) nx = queue_slice_raw(slices, sl + nw);
        SliceWords cur;
        queue_load(I, S, lane, cur);
        queue_eval<TIE>(I, S, cur, sp, lane, sweep, seed, r, dE, my, e6);
    }
}

// A wavefront's first slice of a phase, loaded before the barrier that
// opens the phase (couplings and fields are read-only).
struct QueueCarry {
    Slice S;
    SliceWords W;
    bool valid;
};

// One colour phase of a workgroup item: the wavefront's first slice comes
// loaded in `cy`, the rest as in queue_phase.
template <bool TIE>
__device__ __forceinline__ void queue_phase_wg(const InstDev& I, const Slice* slices, int s_lo, int s_hi,
                                               int8_t* __restrict__ sp, int w, int nw, int lane, uint32_t sweep,
                                               uint64_t seed, uint32_t r, long long& dE, int& my, long long& e6,
                                               const QueueCarry& cy)
{
    if (!cy.valid) return;
    int sl = __builtin_amdgcn_readfirstlane(s_lo + w);
    q_v4 nx = {0u, 0u, 0u, 0u};
    if (sl + nw < s_hi) nx = queue_slice_raw(slices, sl + nw);
    queue_eval<TIE>(I, cy.S, cy.W, sp, lane, sweep, seed, r, dE, my, e6);
    for (sl += nw; sl < s_hi; sl += nw) {
        asm volatile("" : "+s"(nx.x), "+s"(nx.y), "+s"(nx.z), "+s"(nx.w));
        const Slice S = queue_unpack(nx);
        if (sl + nw < s_hi) nx = queue_slice_raw(slices, sl + nw);
        SliceWords cur;
        queue_load(I, S, lane, cur);
        queue_eval<TIE>(I, S, cur, sp, lane, sweep, seed, r, dE, my, e6);
    }
}

// Workgroup barrier that orders LDS only: device-memory loads issued before
// it (the next phase's first slice) stay in flight across it.
__device__ __forceinline__ void queue_lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// e6: -6 E of the last sweep's fields, exact when that sweep flipped nothing.
__device__ __forceinline__ void queue_finish(const InstTab& Q, int r, long long dE, long long e6, int nflip,
                                             int performed, int lastflip, int T, int until_conv,
                                             RepState* __restrict__ rs, CallStats* __restrict__ cs)
{
    RepState* st = rs + Q.rep_base + r;
    if (performed > 0 && lastflip < performed) st->E = -e6 / 6;
    else st->E += dE;
    st->flips += nflip;
    st->sweeps += performed;
    st->lastflip = lastflip;
    const bool conv = until_conv && lastflip < performed;
    if (conv) st->converged = 1;
    atomicAdd(&cs->attempts, (unsigned long long)performed * (unsigned long long)Q.I.n);
    atomicAdd(&cs->flips, (unsigned long long)nflip);
    atomicMax(&cs->sweeps_max, (unsigned long long)performed);
    if (until_conv && !conv) atomicAdd(&cs->unconverged, 1ull);
}

template <bool TIE>
__global__ __launch_bounds__(kBatThreads) void k_queue(const InstTab* __restrict__ tab, const int32_t* __restrict__ ctab,
                                                       const QueueItem* __restrict__ items, int n_big, int n_items,
                                                       uint32_t* __restrict__ counters, int wave_lds,
                                                       RepState* __restrict__ rs, CallStats* __restrict__ cs, int T,
                                                       uint64_t seed, int until_conv)
{
    extern __shared__ uint64_t lds64[];
    int8_t* lds = reinterpret_cast<int8_t*>(lds64);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    __shared__ int s_item, s_any[3];
    // ---- large items: the whole workgroup on one replica
    for (;;) {
        if (tid == 0) s_item = (int)atomicAdd(&counters[0], 1u);
        __syncthreads();
        const int q = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (q >= n_big) break;
        const QueueItem it = items[q];
        const InstTab& Q = tab[it.inst];
        const InstDev& I = Q.I;
        int8_t* gsp = Q.spins + (int64_t)it.r * Q.spin_stride;
        const RepState* st0 = rs + Q.rep_base + it.r;
        const bool frozen = st0->converged != 0;
        if (frozen) continue;
        const uint32_t base = (uint32_t)st0->sweeps;
        for (int k = tid; k < I.n; k += kBatThreads) lds[k] = gsp[k];
        if (tid < 3) s_any[tid] = 0;
        __syncthreads();
        // the instance arrays and slice table in scalar registers
        InstDev J = I;
        J.nbr = queue_uniform(I.nbr);
        J.ta = queue_uniform(I.ta);
        J.tb = queue_uniform(I.tb);
        J.h = queue_uniform(I.h);
        J.ext = queue_uniform(I.ext);
        const Slice* sls = queue_uniform(I.slices);
        const int C = Q.C;
        const int32_t* ct = ctab + Q.ctab_off;
        // this wavefront's first slice of colour 0
        QueueCarry cy;
        {
            const int sl0 = __builtin_amdgcn_readfirstlane(ct[0] + wave);
            cy.valid = sl0 < ct[1];
            if (cy.valid) {
                cy.S = queue_unpack(queue_slice_raw(sls, sl0));
                queue_load(J, cy.S, lane, cy.W);
            }
        }
        long long dE = 0, e6 = 0;
        int nflip = 0, performed = 0, lastflip = 0;
        for (int t = 0; t < T; ++t) {
            int my = 0;
            e6 = 0;
            for (int c = 0; c < C; ++c) {
                // the descriptor of this wavefront's first slice of the next
                // phase, read while this phase runs
                const int cn = c + 1 < C ? c + 1 : 0;
                const int sln = __builtin_amdgcn_readfirstlane(ct[cn] + wave);
                const bool nval = sln < ct[cn + 1];
                q_v4 nraw = {0u, 0u, 0u, 0u};
                if (nval) nraw = queue_slice_raw(sls, sln);
                queue_phase_wg<TIE>(J, sls, ct[c], ct[c + 1], lds, wave, kBatWaves, lane, base + t, seed,
                                    (uint32_t)it.r, dE, my, e6, cy);
                // that slice's words, in flight across the barrier
                asm volatile("" : "+s"(nraw.x), "+s"(nraw.y), "+s"(nraw.z), "+s"(nraw.w));
                cy.valid = nval;
                if (nval) {
                    cy.S = queue_unpack(nraw);
                    queue_load(J, cy.S, lane, cy.W);
                }
                if (c + 1 < C) {
                    queue_lds_barrier();
                } else {
                    // the sweep's last barrier also tells whether it flipped
                    // anything: slot t % 3 is set before the barrier and read
                    // after it; slot (t + 2) % 3 is cleared for sweep t + 2,
                    // after every read of it (sweep t - 1) and a barrier before
                    // any write of it
                    if (__ballot(my != 0) != 0 && lane == 0) s_any[t % 3] = 1;
                    queue_lds_barrier();
                }
            }
            nflip += my;
            performed = t + 1;
            const bool tot = s_any[t % 3] != 0;
            if (tid == 0) s_any[(t + 2) % 3] = 0;
            if (tot) lastflip = t + 1;
            if (until_conv && !tot) break;
        }
        for (int k = tid; k < I.n; k += kBatThreads) gsp[k] = lds[k];
        // fold the workgroup's dE, energy sum and flips
        long long wd = dE, we = e6;
        int wf = nflip;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            wd += __shfl_xor(wd, off, 64);
            we += __shfl_xor(we, off, 64);
            wf += __shfl_xor(wf, off, 64);
        }
        __shared__ long long pd[kBatWaves], pe[kBatWaves];
        __shared__ int pf[kBatWaves];
        if (lane == 0) {
            pd[wave] = wd;
            pe[wave] = we;
            pf[wave] = wf;
        }
        __syncthreads();
        if (tid == 0) {
            long long a = 0, e = 0;
            int b = 0;
            for (int w = 0; w < kBatWaves; ++w) {
                a += pd[w];
                e += pe[w];
                b += pf[w];
            }
            queue_finish(Q, it.r, a, e, b, performed, lastflip, T, until_conv, rs, cs);
        }
        __syncthreads();
    }
    // ---- small items: one wavefront per replica, 16 at a time
    int8_t* wl = lds + wave * wave_lds;
    for (;;) {
        if (tid == 0) s_item = n_big + (int)atomicAdd(&counters[1], (unsigned)kBatWaves);
        __syncthreads();
        const int q0 = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (q0 >= n_items) break;
        const int q = __builtin_amdgcn_readfirstlane(q0 + wave);
        if (q < n_items) {
            const QueueItem it = items[q];
            const InstTab& Q = tab[it.inst];
            const InstDev& I = Q.I;
            int8_t* gsp = Q.spins + (int64_t)it.r * Q.spin_stride;
            const RepState* st0 = rs + Q.rep_base + it.r;
            if (!st0->converged) {
                const uint32_t base = (uint32_t)st0->sweeps;
                for (int k = lane; k < I.n; k += 64) wl[k] = gsp[k];
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                long long dE = 0, e6 = 0;
                int nflip = 0, performed = 0, lastflip = 0;
                for (int t = 0; t < T; ++t) {
                    int my = 0;
                    e6 = 0;
                    for (int c = 0; c < Q.C; ++c) {
                        queue_phase<TIE>(I, I.slices, ctab[Q.ctab_off + c], ctab[Q.ctab_off + c + 1], wl, 0, 1, lane,
                                         base + t, seed, (uint32_t)it.r, dE, my, e6);
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                        __builtin_amdgcn_wave_barrier();
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    }
                    nflip += my;
                    performed = t + 1;
                    int tot = my;
#pragma unroll
                    for (int off = 32; off > 0; off >>= 1) tot += __shfl_xor(tot, off, 64);
                    if (tot) lastflip = t + 1;
                    if (until_conv && tot == 0) break;
                }
                for (int k = lane; k < I.n; k += 64) gsp[k] = wl[k];
                long long wd = dE, we = e6;
                int wf = nflip;
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) {
                    wd += __shfl_xor(wd, off, 64);
                    we += __shfl_xor(we, off, 64);
                    wf += __shfl_xor(wf, off, 64);
                }
                if (lane == 0) queue_finish(Q, it.r, wd, we, wf, performed, lastflip, T, until_conv, rs, cs);
            }
        }
        __syncthreads();
    }
}


int queue_max_blocks(size_t lds)
{
    const void* kern = (const void*)k_queue<true>;
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

hipError_t launch_queue(const InstTab* tab, const int32_t* ctab, const QueueItem* items, int n_big, int n_items,
                        uint32_t* counters, int wave_lds, size_t lds, int grid, RepState* rs, CallStats* cs, int T,
                        uint64_t seed, int rule, int until_conv, hipStream_t st)
{
    const void* kern = rule == 1 ? (const void*)k_queue<true> : (const void*)k_queue<false>;
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (rule == 1)
        hipLaunchKernelGGL(k_queue<true>, dim3(grid), dim3(kBatThreads), lds, st, tab, ctab, items, n_big, n_items,
                           counters, wave_lds, rs, cs, T, seed, until_conv);
    else
        hipLaunchKernelGGL(k_queue<false>, dim3(grid), dim3(kBatThreads), lds, st, tab, ctab, items, n_big, n_items,
                           counters, wave_lds, rs, cs, T, seed, until_conv);
    return hipGetLastError();
}

}  // namespace sg
