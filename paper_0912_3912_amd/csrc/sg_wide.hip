// sg_wide.hip -- the colour phase and the energy of instances in the wide
// form (sg_layout.h: any int32 coupling, field and hyper-coupling value, with
// |h_i| + sum|J_ij| + sum|K| < 2^31 per spin; large sizes and restart counts).
//
// The arithmetic is that of the packed kernels in sg_kernels.hip: the local
// field f_i = h_i + sum_j J_ij s_j + sum_(j,k) K_ijk s_j s_k (every partial
// sum is bounded by the per-spin limit, so int32 holds it), the move cost
// dE_i = 2 s_i f_i (int64: it can reach 2^32), the rule (GREEDY: dE_i < 0;
// GREEDY_TIE: also dE_i == 0 with the Philox bit of (spin, sweep, instance,
// restart)), and energies in int64 with every edge and triple counted once
// (Sec. II eq. (1), Sec. VI eq. (5); move of Sec. IV).  Replicas are spread
// over the grid's y dimension in chunks of at most 65535.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "sg_device.h"
#include "sg_launch.h"
#include "sg_layout.h"

namespace sg {

namespace {

constexpr int kWideThreads = kSlice * kPhaseWaves;
constexpr int kMaxGridY = 65535;

__device__ __forceinline__ long long wide_wave_sum(long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <bool TRI>
__device__ __forceinline__ int32_t wide_field(const WideDev& I, const WSlice& S, int lane, int i,
                                              const int8_t* __restrict__ s)
{
    int32_t f = I.h[i];
    const uint32_t* pn = I.nbr + S.ebase + lane;
    const int32_t* pj = I.J + S.ebase + lane;
    const uint32_t ew = S.ew;
    uint32_t k = 0;
    // four couplings and their partners' spins in flight at a time
    for (; k + 4 <= ew; k += 4) {
        const uint32_t j0 = pn[(k + 0) * kSlice], j1 = pn[(k + 1) * kSlice];
        const uint32_t j2 = pn[(k + 2) * kSlice], j3 = pn[(k + 3) * kSlice];
        const int32_t c0 = pj[(k + 0) * kSlice], c1 = pj[(k + 1) * kSlice];
        const int32_t c2 = pj[(k + 2) * kSlice], c3 = pj[(k + 3) * kSlice];
        f += c0 * s[j0];
        f += c1 * s[j1];
        f += c2 * s[j2];
        f += c3 * s[j3];
    }
    for (; k < ew; ++k) f += pj[k * kSlice] * s[pn[k * kSlice]];
    if (TRI) {
        const uint32_t* pa = I.ta + S.tbase + lane;
        const uint32_t* pb = I.tb + S.tbase + lane;
        const int32_t* pk = I.K + S.tbase + lane;
        for (uint32_t q = 0; q < S.tw; ++q) f += pk[q * kSlice] * s[pa[q * kSlice]] * s[pb[q * kSlice]];
    }
    return f;
}

__device__ __forceinline__ bool wide_active(const RepState* st, int t_rel, int until_conv)
{
    const int conv = __hip_atomic_load(&st->converged, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (conv) return false;
    if (!until_conv || t_rel == 0) return true;
    const int lf = __hip_atomic_load(&st->lastflip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return lf >= t_rel;
}

// One colour phase of one wide instance: grid = (ceil(slices_c / 4), replicas
// of this chunk), replica r = r0 + blockIdx.y; per-block accumulators as in
// k_phase (slot r * nslots + blockIdx.x holds dE and the flip count).
template <bool TIE, bool TRI>
__global__ __launch_bounds__(kWideThreads) void k_wide_phase(WideDev I, int8_t* __restrict__ spins, int64_t stride,
                                                             RepState* __restrict__ rs, int64_t* __restrict__ acc,
                                                             int nslots, int slice0, int nslice_c, int t_local,
                                                             const int32_t* __restrict__ t_base, uint64_t seed,
                                                             int until_conv, int r0)
{
    const int t_rel = t_local + (t_base ? *t_base : 0);
    const int r = r0 + (int)blockIdx.y;
    RepState* st = rs + r;
    if (!wide_active(st, t_rel, until_conv)) return;
    int8_t* s = spins + (int64_t)r * stride;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int sl = blockIdx.x * kPhaseWaves + wave;
    long long dflip = 0;
    bool flip = false;
    if (sl < nslice_c) {
        const WSlice S = I.slices[slice0 + sl];
        if ((uint32_t)lane < S.rows) {
            const int i = (int)S.row0 + lane;
            const int32_t f = wide_field<TRI>(I, S, lane, i, s);
            const int si = s[i];
            const long long d = 2LL * si * (long long)f;
            flip = d < 0;
            if (TIE && d == 0) {
                const uint32_t sweep = (uint32_t)(st->sweeps + t_rel);
                flip = rng_bit(seed, I.ext[i], sweep, I.instance_id, (uint32_t)r) != 0;
            }
            if (flip) {
                s[i] = (int8_t)(-si);
                dflip = d;
            }
        }
    }
    const int nf = (int)__popcll(__ballot(flip));
    const long long dsum = wide_wave_sum(dflip);
    __shared__ long long part_d[kPhaseWaves];
    __shared__ int part_f[kPhaseWaves];
    if (lane == 0) {
        part_d[wave] = dsum;
        part_f[wave] = nf;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        long long td = 0;
        int tf = 0;
#pragma unroll
        for (int w = 0; w < kPhaseWaves; ++w) {
            td += part_d[w];
            tf += part_f[w];
        }
        if (tf) {
            int64_t* a = acc + 2 * ((int64_t)r * nslots + blockIdx.x);
            a[0] += td;
            a[1] += tf;
            if (until_conv &&
                __hip_atomic_load(&st->lastflip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < t_rel + 1)
                __hip_atomic_store(&st->lastflip, t_rel + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Energy of a wide instance: every row i adds h_i s_i + sum_{j > i} J s_i s_j
// + sum_{a > i, b > i} K s_i s_a s_b, so each edge and triple is counted once;
// grid = (nslots, replicas of this chunk); slots[r * nslots + b] = -(block sum).
__global__ __launch_bounds__(kWideThreads) void k_wide_energy(WideDev I, const int8_t* __restrict__ spins,
                                                              int64_t stride, int64_t* __restrict__ slots, int nslots,
                                                              int r0)
{
    const int r = r0 + (int)blockIdx.y;
    const int8_t* s = spins + (int64_t)r * stride;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    long long acc = 0;
    for (int sl = blockIdx.x * kPhaseWaves + wave; sl < I.nslices; sl += nslots * kPhaseWaves) {
        const WSlice S = I.slices[sl];
        if ((uint32_t)lane < S.rows) {
            const uint32_t i = S.row0 + lane;
            const int si = s[i];
            long long e = (long long)I.h[i] * si;
            const uint32_t* pn = I.nbr + S.ebase + lane;
            const int32_t* pj = I.J + S.ebase + lane;
            for (uint32_t k = 0; k < S.ew; ++k) {
                const uint32_t j = pn[k * kSlice];
                if (j > i) e += (long long)pj[k * kSlice] * si * s[j];
            }
            if (I.has_tri) {
                const uint32_t* pa = I.ta + S.tbase + lane;
                const uint32_t* pb = I.tb + S.tbase + lane;
                const int32_t* pk = I.K + S.tbase + lane;
                for (uint32_t k = 0; k < S.tw; ++k) {
                    const uint32_t a = pa[k * kSlice], b = pb[k * kSlice];
                    if (a > i && b > i) e += (long long)pk[k * kSlice] * si * s[a] * s[b];
                }
            }
            acc += e;
        }
    }
    acc = wide_wave_sum(acc);
    __shared__ long long part[kPhaseWaves];
    if (lane == 0) part[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long t = 0;
        for (int w = 0; w < kPhaseWaves; ++w) t += part[w];
        slots[(int64_t)r * nslots + blockIdx.x] = -t;
    }
}

}  // namespace

hipError_t launch_wide_phase(const WideDev& I, int8_t* spins, int64_t stride, RepState* rs, int R, int64_t* acc,
                             int nslots, int slice0, int nslice_c, int t_rel, uint64_t seed, int rule, int until_conv,
                             hipStream_t st, const int32_t* t_base)
{
    const bool tie = rule == 1, tri = I.has_tri != 0;
    const unsigned gx = (unsigned)((nslice_c + kPhaseWaves - 1) / kPhaseWaves);
    if (gx == 0) return hipSuccess;
    for (int r0 = 0; r0 < R; r0 += kMaxGridY) {
        const dim3 grid(gx, (unsigned)std::min(kMaxGridY, R - r0));
#define SG_WIDE_LAUNCH(TIE_, TRI_)                                                                                 \
    hipLaunchKernelGGL((k_wide_phase<TIE_, TRI_>), grid, dim3(kWideThreads), 0, st, I, spins, stride, rs, acc,    \
                       nslots, slice0, nslice_c, t_rel, t_base, seed, until_conv, r0)
        if (tie && tri) SG_WIDE_LAUNCH(true, true);
        else if (tie) SG_WIDE_LAUNCH(true, false);
        else if (tri) SG_WIDE_LAUNCH(false, true);
        else SG_WIDE_LAUNCH(false, false);
#undef SG_WIDE_LAUNCH
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_wide_energy(const WideDev& I, const int8_t* spins, int64_t stride, int R, int64_t* slots,
                              int nslots, RepState* rs, int64_t* out, hipStream_t st)
{
    for (int r0 = 0; r0 < R; r0 += kMaxGridY) {
        const dim3 grid((unsigned)nslots, (unsigned)std::min(kMaxGridY, R - r0));
        hipLaunchKernelGGL(k_wide_energy, grid, dim3(kWideThreads), 0, st, I, spins, stride, slots, nslots, r0);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return launch_reduce_energy(slots, nslots, R, rs, out, st);
}

}  // namespace sg
