// sg_dense.hip -- dense hyper-Ising instances (Sec. VI eq. (5)): at most 64
// spins, couplings over any set of spins with int64 coefficients, e.g. the
// factoring hypergraphs of eqs. (6)-(8), whose terms reach four spins and whose
// coefficients outgrow the sparse kernels' int8/int32 ranges.
//
// One lane per replica, 64 replicas of one instance per wavefront (an item =
// instance, first restart, count).  A lane holds its spins as a 64-bit word
// (bit i set when s_i = -1); the product of the spins of a term t is
// (-1)^popcount(state & mask_t), so a term costs a few integer instructions
// and the term lists, the same for every lane, are read with scalar loads.
//   k_dense_init    random start (the Philox start rule of the sparse path),
//                   energy, replica state reset
//   k_dense_energy  energies of the stored spins
//   k_dense_sweep   colour-ordered sweeps, GREEDY / GREEDY_TIE, the stopping
//                   rule of the sparse path
//   k_dense_fm      the pass-based search (max-gain moves, locking,
//                   hill-climbing, best state of a pass kept); the gains live
//                   in LDS as [spin][lane] and a move updates only the gains of
//                   the spins that share a term with it: flipping s_p changes
//                   the gain of every other member j of a term t by
//                   4 coef_t prod_{k in t} s_k (the product before the flip)
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sg_device.h"
#include "sg_launch.h"
#include "sg_layout.h"

namespace sg {

constexpr int kDenseThreads = 256;
constexpr int kDenseWaves = kDenseThreads / 64;

__device__ __forceinline__ long long dense_term(uint64_t state, uint64_t m, long long c)
{
    return (__popcll(state & m) & 1) ? -c : c;
}

__device__ __forceinline__ long long dense_energy_of(const DenseTab& D, uint64_t state)
{
    long long E = 0;
    for (int t = 0; t < D.nterms; ++t) E -= dense_term(state, D.tmask[t], D.tcoef[t]);
    return E;
}

// f_i = sum over terms holding i of coef * (product of the other members)
__device__ __forceinline__ long long dense_field(const DenseTab& D, uint64_t state, int i)
{
    long long f = 0;
    for (int e = D.dstart[i]; e < D.dstart[i + 1]; ++e) f += dense_term(state, D.dmask[e], D.dcoef[e]);
    return f;
}

__device__ __forceinline__ uint64_t dense_load(const DenseTab& D, int r)
{
    const int8_t* s = D.spins + D.spin_stride * r;
    uint64_t state = 0;
    for (int i = 0; i < D.n; ++i)
        if (s[i] < 0) state |= 1ull << i;
    return state;
}

__device__ __forceinline__ void dense_store(const DenseTab& D, int r, uint64_t state)
{
    int8_t* s = D.spins + D.spin_stride * r;
    for (int i = 0; i < D.n; ++i) s[i] = (int8_t)(((state >> i) & 1ull) ? -1 : 1);
}

// call totals: one atomic per block
__device__ __forceinline__ void dense_totals(CallStats* cs, long long att, long long flips, long long sweeps,
                                             int unconv)
{
    __shared__ unsigned long long b[4];
    if (threadIdx.x < 4) b[threadIdx.x] = 0;
    __syncthreads();
    if (att) atomicAdd(&b[0], (unsigned long long)att);
    if (flips) atomicAdd(&b[1], (unsigned long long)flips);
    if (sweeps) atomicMax(&b[2], (unsigned long long)sweeps);
    if (unconv) atomicAdd(&b[3], 1ull);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (b[0]) atomicAdd(&cs->attempts, b[0]);
        if (b[1]) atomicAdd(&cs->flips, b[1]);
        if (b[2]) atomicMax(&cs->sweeps_max, b[2]);
        if (b[3]) atomicAdd(&cs->unconverged, b[3]);
    }
}

__global__ __launch_bounds__(kDenseThreads) void k_dense_init(const DenseTab* __restrict__ tabs,
                                                              const BlockItem* __restrict__ items, int nitems,
                                                              RepState* __restrict__ rs, uint64_t seed)
{
    const int item = blockIdx.x * kDenseWaves + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (item >= nitems) return;
    const BlockItem it = items[item];
    if (lane >= it.nr) return;
    const DenseTab D = tabs[it.inst];
    const int r = it.r0 + lane;
    uint64_t state = 0;
    for (int i = 0; i < D.n; ++i)
        if (rng_bit(seed, (uint32_t)i, 0xFFFFFFFFu, D.instance_id, (uint32_t)r)) state |= 1ull << i;
    dense_store(D, r, state);
    RepState z;
    z.E = dense_energy_of(D, state);
    z.flips = 0;
    z.sweeps = 0;
    z.lastflip = 0;
    z.converged = 0;
    rs[D.rep_base + r] = z;
}

__global__ __launch_bounds__(kDenseThreads) void k_dense_energy(const DenseTab* __restrict__ tabs,
                                                                const BlockItem* __restrict__ items, int nitems,
                                                                int64_t* __restrict__ out)
{
    const int item = blockIdx.x * kDenseWaves + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (item >= nitems) return;
    const BlockItem it = items[item];
    if (lane >= it.nr) return;
    const DenseTab D = tabs[it.inst];
    const int r = it.r0 + lane;
    out[D.rep_base + r] = dense_energy_of(D, dense_load(D, r));
}

template <bool TIE>
__global__ __launch_bounds__(kDenseThreads) void k_dense_sweep(const DenseTab* __restrict__ tabs,
                                                               const BlockItem* __restrict__ items, int nitems,
                                                               RepState* __restrict__ rs, CallStats* __restrict__ cs,
                                                               int max_sweeps, int until_conv, uint64_t seed)
{
    const int item = blockIdx.x * kDenseWaves + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    long long att = 0, nfl = 0, nsw = 0;
    int unconv = 0;
    if (item < nitems) {
        const BlockItem it = items[item];
        const DenseTab D = tabs[it.inst];
        const int r = it.r0 + lane;
        const bool mine = lane < it.nr;
        RepState* st = rs + D.rep_base + (mine ? r : it.r0);
        bool active = mine && !st->converged;
        uint64_t state = mine ? dense_load(D, r) : 0;
        long long E = mine ? st->E : 0;
        const long long sw0 = mine ? st->sweeps : 0;
        int done = 0;
        // every lane walks the same spins in the same order (wave-uniform loops)
        for (int t = 0; t < max_sweeps && __ballot(active); ++t) {
            const uint32_t sweep = (uint32_t)(sw0 + t);
            int F = 0;
            for (int k = 0; k < D.n; ++k) {
                const int i = D.order[k];
                const long long f = dense_field(D, state, i);
                const long long d = ((state >> i) & 1ull) ? -2 * f : 2 * f;
                bool flip = d < 0;
                if (TIE && d == 0 && active)
                    flip = rng_bit(seed, (uint32_t)i, sweep, D.instance_id, (uint32_t)r) != 0;
                if (active && flip) {
                    state ^= 1ull << i;
                    E += d;
                    ++F;
                }
            }
            if (active) {
                ++done;
                nfl += F;
                if (until_conv && F == 0) active = false;
            }
        }
        if (mine && !st->converged) {
            dense_store(D, r, state);
            st->E = E;
            st->sweeps += done;
            st->flips += nfl;
            const bool conv = until_conv && done > 0 && !active;
            if (conv) st->converged = 1;
            att = (long long)done * D.n;
            nsw = done;
            unconv = (until_conv && !conv) ? 1 : 0;
        } else {
            nfl = 0;
        }
    }
    dense_totals(cs, att, nfl, nsw, unconv);
}

__global__ __launch_bounds__(kDenseThreads) void k_dense_fm(const DenseTab* __restrict__ tabs,
                                                            const BlockItem* __restrict__ items, int nitems, int nmax,
                                                            RepState* __restrict__ rs, CallStats* __restrict__ cs,
                                                            int max_passes, int until_conv)
{
    extern __shared__ long long dgain[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int item = blockIdx.x * kDenseWaves + wave;
    long long att = 0, kept = 0, npass = 0;
    int unconv = 0;
    if (item < nitems) {
        const BlockItem it = items[item];
        const DenseTab D = tabs[it.inst];
        const int n = D.n;
        long long* G = dgain + (size_t)wave * nmax * 64;  // G[i * 64 + lane]
        const int r = it.r0 + lane;
        const bool mine = lane < it.nr;
        RepState* st = rs + D.rep_base + (mine ? r : it.r0);
        bool active = mine && !st->converged;
        uint64_t state = mine ? dense_load(D, r) : 0;
        long long E = mine ? st->E : 0;
        int done = 0;
        for (int pass = 0; pass < max_passes && __ballot(active); ++pass) {
            for (int i = 0; i < n; ++i) {
                const long long f = dense_field(D, state, i);
                G[i * 64 + lane] = ((state >> i) & 1ull) ? 2 * f : -2 * f;
            }
            // the wavefront runs the pass for all lanes; a lane that has
            // stopped gets its state back at the end of the pass
            const uint64_t start = state;
            uint64_t locked = 0, best = state;
            const long long Estart = E;
            long long Elow = E;
            int best_len = 0;
            for (int step = 0; step < n; ++step) {
                int pick = -1;
                long long pg = 0;
                for (int i = 0; i < n; ++i) {
                    if ((locked >> i) & 1ull) continue;
                    const long long g = G[i * 64 + lane];
                    if (pick < 0 || g > pg) {
                        pick = i;
                        pg = g;
                    }
                }
                const uint64_t old = state;
                const uint64_t pb = 1ull << pick;
                state ^= pb;
                locked |= pb;
                E -= pg;
                for (int e = D.dstart[pick]; e < D.dstart[pick + 1]; ++e) {
                    uint64_t m = D.dmask[e];
                    const long long delta = 4 * dense_term(old, m | pb, D.dcoef[e]);
                    while (m) {
                        const int j = __builtin_ctzll(m);
                        m &= m - 1;
                        G[j * 64 + lane] += delta;
                    }
                }
                if (E < Elow) {
                    Elow = E;
                    best = state;
                    best_len = step + 1;
                }
            }
            if (active) {
                state = best;
                E = Elow;
                ++done;
                kept += best_len;
                if (until_conv && !(Elow < Estart)) active = false;
            } else {
                state = start;
                E = Estart;
            }
        }
        if (mine && !st->converged) {
            dense_store(D, r, state);
            st->E = E;
            st->sweeps += done;
            st->flips += kept;
            const bool conv = until_conv && done > 0 && !active;
            if (conv) st->converged = 1;
            att = (long long)done * n;
            npass = done;
            unconv = (until_conv && !conv) ? 1 : 0;
        } else {
            kept = 0;
        }
    }
    dense_totals(cs, att, kept, npass, unconv);
}

// ---------------------------------------------------------------------------

hipError_t launch_dense_init(const DenseTab* tabs, const BlockItem* items, int nitems, RepState* rs, uint64_t seed,
                             hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_dense_init, dim3((nitems + kDenseWaves - 1) / kDenseWaves), dim3(kDenseThreads), 0, st, tabs,
                       items, nitems, rs, seed);
    return hipGetLastError();
}

hipError_t launch_dense_energy(const DenseTab* tabs, const BlockItem* items, int nitems, int64_t* out, hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_dense_energy, dim3((nitems + kDenseWaves - 1) / kDenseWaves), dim3(kDenseThreads), 0, st,
                       tabs, items, nitems, out);
    return hipGetLastError();
}

hipError_t launch_dense_run(const DenseTab* tabs, const BlockItem* items, int nitems, int nmax, RepState* rs,
                            CallStats* cs, int rule, int max_sweeps, int until_conv, uint64_t seed, hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    const dim3 grid((nitems + kDenseWaves - 1) / kDenseWaves);
    if (rule == 2) {
        const size_t lds = (size_t)kDenseWaves * nmax * 64 * 8;
        hipError_t e = hipFuncSetAttribute((const void*)k_dense_fm, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_dense_fm, grid, dim3(kDenseThreads), lds, st, tabs, items, nitems, nmax, rs, cs,
                           max_sweeps, until_conv);
    } else if (rule == 1) {
        hipLaunchKernelGGL(k_dense_sweep<true>, grid, dim3(kDenseThreads), 0, st, tabs, items, nitems, rs, cs,
                           max_sweeps, until_conv, seed);
    } else {
        hipLaunchKernelGGL(k_dense_sweep<false>, grid, dim3(kDenseThreads), 0, st, tabs, items, nitems, rs, cs,
                           max_sweeps, until_conv, seed);
    }
    return hipGetLastError();
}

}  // namespace sg
