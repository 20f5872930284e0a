// sg_kernels.hip -- HIP kernels for gfx950 (wave64) and their launchers.
//
// The hot path is the colour phase: every spin i of one colour computes its
// local field f_i = h_i + sum_j J_ij s_j + sum_(j,k) K_ijk s_j s_k, its move
// cost dE_i = 2 s_i f_i (Sec. IV: the move's gain is -dE_i), decides the move
// (GREEDY: dE_i < 0; GREEDY_TIE: also dE_i == 0 with an RNG bit) and flips.
// The spins of one colour share no energy term (proper colouring of the
// primal graph), so deciding them all at once equals deciding them one by
// one.  Energy changes and flip counts are reduced per wavefront with
// ballot/popcount and butterfly shuffles, then per block through LDS, and
// accumulated per block in its own slot (no atomics on the hot path).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sg_device.h"
#include "sg_launch.h"
#include "sg_layout.h"

namespace sg {

__device__ __forceinline__ int wave_sum_i32(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ long long wave_sum_i64(long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ int coupling_j(uint32_t w) { return (int)(int8_t)(w & 0xffu); }

// ---------------------------------------------------------------------------
// Utility kernels

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint64_t count, uint32_t v)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Energy, Sec. II eq. (1) / Sec. VI eq. (5): each row i adds
// h_i s_i + sum_{j > i} J s_i s_j + sum_{i < a, i < b} K s_i s_a s_b, so every
// edge and triple is counted once (at its smallest internal index).
// grid = (nslots, R); block b walks slices b*4+w, b*4+w + 4*nslots, ...
// slots[r*nslots + b] = -(block sum).
__global__ __launch_bounds__(kPhaseThreads) void k_energy(InstDev I, const int8_t* __restrict__ spins,
                                                          int64_t stride, int64_t* __restrict__ slots,
                                                          int nslots)
{
    const int r = blockIdx.y;
    const int8_t* s = spins + r * stride;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    long long acc = 0;
    for (int sl = blockIdx.x * kPhaseWaves + wave; sl < I.nslices; sl += nslots * kPhaseWaves) {
        const Slice S = I.slices[sl];
        if (lane < S.rows) {
            const int i = S.row0 + lane;
            const int si = s[i];
            int e = I.h[i] * si;
            const uint32_t* p = I.nbr + S.ebase + lane;
            for (int k = 0; k < S.ew; ++k) {
                const uint32_t w = p[k * kSlice];
                const int j = (int)(w >> 8);
                if (j > i) e += coupling_j(w) * si * s[j];
            }
            if (I.has_tri) {
                const uint32_t* pa = I.ta + S.tbase + lane;
                const uint32_t* pb = I.tb + S.tbase + lane;
                for (int k = 0; k < S.tw; ++k) {
                    const uint32_t wa = pa[k * kSlice];
                    const int a = (int)(wa >> 8);
                    const int b = (int)pb[k * kSlice];
                    if (a > i && b > i) e += coupling_j(wa) * si * s[a] * s[b];
                }
            }
            acc += e;
        }
    }
    acc = wave_sum_i64(acc);
    __shared__ long long part[kPhaseWaves];
    if (lane == 0) part[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long t = 0;
        for (int w = 0; w < kPhaseWaves; ++w) t += part[w];
        slots[(int64_t)r * nslots + blockIdx.x] = -t;
    }
}

// out[r] (or rs[r].E when to_state) = sum of slots[r*nslots ...]; one block per replica.
__global__ void k_reduce_energy(const int64_t* __restrict__ slots, int nslots, RepState* __restrict__ rs,
                                int64_t* __restrict__ out)
{
    const int r = blockIdx.x;
    long long acc = 0;
    for (int k = threadIdx.x; k < nslots; k += blockDim.x) acc += slots[(int64_t)r * nslots + k];
    acc = wave_sum_i64(acc);
    __shared__ long long part[16];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) part[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long t = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += part[w];
        if (out) out[r] = t;
        else rs[r].E = t;
    }
}

// Start of a call: clear the per-block accumulators and the lastflip marks.
__global__ void k_begin(RepState* __restrict__ rs, int R, int64_t* __restrict__ acc, int64_t nacc)
{
    const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = tid; k < nacc; k += stride) acc[k] = 0;
    for (int64_t r = tid; r < R; r += stride) rs[r].lastflip = 0;
}

__device__ __forceinline__ bool replica_active(const RepState* st, int t_rel, int until_conv)
{
    const int conv = __hip_atomic_load(&st->converged, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (conv) return false;
    if (!until_conv || t_rel == 0) return true;
    const int lf = __hip_atomic_load(&st->lastflip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return lf >= t_rel;
}

// Field of internal row i (lane's row of slice S).
template <bool TRI>
__device__ __forceinline__ int local_field(const InstDev& I, const Slice& S, int lane, int i,
                                           const int8_t* __restrict__ s)
{
    int f = I.h[i];
    const uint32_t* p = I.nbr + S.ebase + lane;
    const int ew = S.ew;
    // up to 16 coupling words, then their partners' spins, in flight together
    constexpr int kPre = 16;
    uint32_t w[kPre];
    int sj[kPre];
#pragma unroll
    for (int k = 0; k < kPre; ++k) w[k] = k < ew ? p[k * kSlice] : 0u;
#pragma unroll
    for (int k = 0; k < kPre; ++k) sj[k] = k < ew ? s[w[k] >> 8] : 0;
#pragma unroll
    for (int k = 0; k < kPre; ++k) f += coupling_j(w[k]) * sj[k];
    for (int k = kPre; k < ew; ++k) {
        const uint32_t w1 = p[k * kSlice];
        f += coupling_j(w1) * s[w1 >> 8];
    }
    if (TRI) {
        const uint32_t* pa = I.ta + S.tbase + lane;
        const uint32_t* pb = I.tb + S.tbase + lane;
        for (int q = 0; q < S.tw; ++q) {
            const uint32_t wa = pa[q * kSlice];
            const uint32_t b = pb[q * kSlice];
            f += coupling_j(wa) * s[wa >> 8] * s[b];
        }
    }
    return f;
}

// Local fields of every spin of every replica (the start of a run over
// maintained fields): grid = (ceil(nslices/4), R).
template <bool TRI>
__global__ __launch_bounds__(kPhaseThreads) void k_fields(InstDev I, const int8_t* __restrict__ spins,
                                                          int64_t stride, int32_t* __restrict__ fields,
                                                          int64_t fstride)
{
    const int r = blockIdx.y;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int sl = blockIdx.x * kPhaseWaves + wave;
    if (sl >= I.nslices) return;
    const Slice S = I.slices[sl];
    if (lane < S.rows) {
        const int i = S.row0 + lane;
        fields[(int64_t)r * fstride + i] = local_field<TRI>(I, S, lane, i, spins + (int64_t)r * stride);
    }
}

// One colour phase of one instance (the plain method): grid = (ceil(slices_c/4), R),
// block = 4 wavefronts, wavefront w of block x handles slice slice0 + 4x + w.
// t_rel = t_local + (*t_base when t_base is not null): graph replays keep the
// launch arguments fixed and advance the base in device memory.
//
// INC (maintained fields, the "only the neighbours' gains change" idea of
// Sec. IV): f_i is read from the replica's field array instead of being
// summed over the couplings, and a spin that flips adds the change of its
// partners' fields, -2 J_ij s_i to f_j and -2 K s_i s_b to f_a for a triple
// (i, a, b), with integer atomics.  Partners have other colours (proper
// colouring), so every field read in a phase is exact; a phase with few
// flips moves a few bytes per spin instead of the coupling stream.
template <bool TIE, bool TRI, bool INC>
__global__ __launch_bounds__(kPhaseThreads) void k_phase(InstDev I, int8_t* __restrict__ spins,
                                                         int64_t stride, RepState* __restrict__ rs,
                                                         int64_t* __restrict__ acc, int nslots,
                                                         int slice0, int nslice_c, int t_local,
                                                         const int32_t* __restrict__ t_base,
                                                         uint64_t seed, int until_conv,
                                                         int32_t* __restrict__ fields, int64_t fstride)
{
    const int t_rel = t_local + (t_base ? *t_base : 0);
    const int r = blockIdx.y;
    RepState* st = rs + r;
    if (!replica_active(st, t_rel, until_conv)) return;
    int8_t* s = spins + (int64_t)r * stride;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int sl = blockIdx.x * kPhaseWaves + wave;
    int dflip = 0;
    bool flip = false;
    if (sl < nslice_c) {
        const Slice S = I.slices[slice0 + sl];
        if (lane < S.rows) {
            const int i = S.row0 + lane;
            int32_t* F = INC ? fields + (int64_t)r * fstride : nullptr;
            const int f = INC ? F[i] : local_field<TRI>(I, S, lane, i, s);
            const int si = s[i];
            const int d = 2 * si * f;
            flip = d < 0;
            if (TIE && d == 0) {
                const uint32_t sweep = (uint32_t)(st->sweeps + t_rel);
                flip = rng_bit(seed, I.ext[i], sweep, I.instance_id, (uint32_t)r) != 0;
            }
            if (flip) {
                s[i] = (int8_t)(-si);
                dflip = d;
                if (INC) {
                    const uint32_t* p = I.nbr + S.ebase + lane;
                    for (int k = 0; k < S.ew; ++k) {
                        const uint32_t w = p[k * kSlice];
                        const int J = coupling_j(w);
                        if (J) atomicAdd(F + (w >> 8), -2 * J * si);
                    }
                    if (TRI) {
                        const uint32_t* pa = I.ta + S.tbase + lane;
                        const uint32_t* pb = I.tb + S.tbase + lane;
                        for (int q = 0; q < S.tw; ++q) {
                            const uint32_t wa = pa[q * kSlice];
                            const int K = coupling_j(wa);
                            if (K) {
                                const int a = (int)(wa >> 8), b = (int)pb[q * kSlice];
                                atomicAdd(F + a, -2 * K * si * s[b]);
                                atomicAdd(F + b, -2 * K * si * s[a]);
                            }
                        }
                    }
                }
            }
        }
    }
    const int nf = (int)__popcll(__ballot(flip));
    const int dsum = wave_sum_i32(dflip);
    __shared__ int part_d[kPhaseWaves], part_f[kPhaseWaves];
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
            // Mark "this sweep flipped" for the stopping rule.  Every writer
            // stores the same value; skip the store once it is visible so
            // that thousands of blocks do not serialise on one word.
            if (until_conv &&
                __hip_atomic_load(&st->lastflip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < t_rel + 1)
                __hip_atomic_store(&st->lastflip, t_rel + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// End of a call, one block per replica: fold the per-block accumulators into
// the replica state, settle the sweep count and the converged flag, add the
// call totals.  T = sweeps launched in this call.  The first accumulator of
// each slot is an energy change, or with `absolute` the slot's share of the
// final energy (then it replaces E of every replica not frozen at entry).
__global__ void k_end(RepState* __restrict__ rs, const int64_t* __restrict__ acc, int nslots, int T,
                      int until_conv, int64_t n, CallStats* __restrict__ cs, int absolute)
{
    const int r = blockIdx.x;
    RepState* st = rs + r;
    long long dE = 0, nf = 0;
    for (int k = threadIdx.x; k < nslots; k += blockDim.x) {
        dE += acc[2 * ((int64_t)r * nslots + k)];
        nf += acc[2 * ((int64_t)r * nslots + k) + 1];
    }
    dE = wave_sum_i64(dE);
    nf = wave_sum_i64(nf);
    __shared__ long long pd[16], pf[16];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        pd[wave] = dE;
        pf[wave] = nf;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    long long td = 0, tf = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
        td += pd[w];
        tf += pf[w];
    }
    int performed = 0;
    int conv = st->converged;
    const int frozen = conv;
    if (!conv) {
        if (until_conv) {
            const int L = st->lastflip;
            if (L >= T) {
                performed = T;
            } else {
                performed = L + 1;
                conv = 1;
            }
        } else {
            performed = T;
        }
    }
    if (!absolute) st->E += td;
    else if (!frozen) st->E = td;
    st->flips += tf;
    st->sweeps += performed;
    st->converged = conv;
    atomicAdd(&cs->attempts, (unsigned long long)((long long)performed * n));
    atomicAdd(&cs->flips, (unsigned long long)tf);
    atomicMax(&cs->sweeps_max, (unsigned long long)performed);
    if (until_conv && !conv) atomicAdd(&cs->unconverged, 1ull);
}

// Any replica still moving after T launched sweeps?  flag must be zero on entry.
__global__ void k_any_active(const RepState* __restrict__ rs, int R, int T, uint32_t* __restrict__ flag)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < R && !rs[r].converged && rs[r].lastflip >= T) *flag = 1u;
}

// Word 0 of Philox4x32-10 for count counters (4 words each), key = seed: the
// generator behind every start and tie decision, exposed for checking.
__global__ void k_philox_word0(const uint32_t* __restrict__ ctr, uint32_t* __restrict__ out, int64_t count,
                               uint64_t seed)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = philox_word0(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], (uint32_t)seed,
                              (uint32_t)(seed >> 32));
}

// Multi-start result per instance: lowest tracked energy, lowest restart on
// ties.  One wavefront per instance: lanes take restarts lane, lane + 64, ...,
// then a butterfly keeps the lexicographically smallest (energy, restart).
__global__ void k_best(const RepState* __restrict__ rs, const int64_t* __restrict__ rep_base,
                       const int32_t* __restrict__ restarts, int ninst, int64_t* __restrict__ Eb,
                       int32_t* __restrict__ rb)
{
    const int q = blockIdx.x * (int)(blockDim.x >> 6) + (int)(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (q >= ninst) return;  // uniform over the wavefront
    const RepState* p = rs + rep_base[q];
    const int R = restarts[q];
    long long e = 0x7FFFFFFFFFFFFFFFll;
    int best = 0x7FFFFFFF;
    for (int r = lane; r < R; r += 64) {
        const long long v = p[r].E;
        if (v < e) {  // restarts rise along a lane: the first of equal energies is kept
            e = v;
            best = r;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const long long e2 = __shfl_xor(e, o, 64);
        const int b2 = __shfl_xor(best, o, 64);
        if (e2 < e || (e2 == e && b2 < best)) {
            e = e2;
            best = b2;
        }
    }
    if (lane == 0) {
        Eb[q] = e;
        rb[q] = best;
    }
}

// ---------------------------------------------------------------------------
// launchers

static unsigned grid1(uint64_t work, unsigned threads, unsigned cap = 65535u)
{
    uint64_t g = (work + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

hipError_t launch_fill_u32(void* p, uint64_t count, uint32_t v, hipStream_t st)
{
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid1(count, 256, 4096)), dim3(256), 0, st, (uint32_t*)p, count, v);
    return hipGetLastError();
}

hipError_t launch_energy(const InstDev& I, const int8_t* spins, int64_t stride, int R, int64_t* slots,
                         int nslots, RepState* rs, int64_t* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_energy, dim3(nslots, R), dim3(kPhaseThreads), 0, st, I, spins, stride, slots, nslots);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_energy, dim3(R), dim3(256), 0, st, (const int64_t*)slots, nslots, rs, out);
    return hipGetLastError();
}

hipError_t launch_reduce_energy(const int64_t* slots, int nslots, int R, RepState* rs, int64_t* out, hipStream_t st)
{
    if (R <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_energy, dim3(R), dim3(256), 0, st, slots, nslots, rs, out);
    return hipGetLastError();
}

hipError_t launch_begin(RepState* rs, int R, int64_t* acc, int64_t nacc, hipStream_t st)
{
    const uint64_t work = (uint64_t)(nacc > R ? nacc : R);
    hipLaunchKernelGGL(k_begin, dim3(grid1(work, 256, 4096)), dim3(256), 0, st, rs, R, acc, nacc);
    return hipGetLastError();
}

hipError_t launch_phase(const InstDev& I, int8_t* spins, int64_t stride, RepState* rs, int R, int64_t* acc,
                        int nslots, int slice0, int nslice_c, int t_rel, uint64_t seed, int rule,
                        int until_conv, hipStream_t st, const int32_t* t_base, int32_t* fields, int64_t fstride)
{
    const dim3 grid((nslice_c + kPhaseWaves - 1) / kPhaseWaves, R);
    const bool tie = rule == 1, tri = I.has_tri != 0;
#define SG_PHASE_LAUNCH(TIE_, TRI_, INC_)                                                                          \
    hipLaunchKernelGGL((k_phase<TIE_, TRI_, INC_>), grid, dim3(kPhaseThreads), 0, st, I, spins, stride, rs, acc,  \
                       nslots, slice0, nslice_c, t_rel, t_base, seed, until_conv, fields, fstride)
    if (fields) {
        if (tie && tri) SG_PHASE_LAUNCH(true, true, true);
        else if (tie) SG_PHASE_LAUNCH(true, false, true);
        else if (tri) SG_PHASE_LAUNCH(false, true, true);
        else SG_PHASE_LAUNCH(false, false, true);
    } else {
        if (tie && tri) SG_PHASE_LAUNCH(true, true, false);
        else if (tie) SG_PHASE_LAUNCH(true, false, false);
        else if (tri) SG_PHASE_LAUNCH(false, true, false);
        else SG_PHASE_LAUNCH(false, false, false);
    }
#undef SG_PHASE_LAUNCH
    return hipGetLastError();
}

hipError_t launch_fields(const InstDev& I, const int8_t* spins, int64_t stride, int R, int32_t* fields, int64_t fstride,
                         hipStream_t st)
{
    const dim3 grid((I.nslices + kPhaseWaves - 1) / kPhaseWaves, R);
    if (I.has_tri)
        hipLaunchKernelGGL((k_fields<true>), grid, dim3(kPhaseThreads), 0, st, I, spins, stride, fields, fstride);
    else
        hipLaunchKernelGGL((k_fields<false>), grid, dim3(kPhaseThreads), 0, st, I, spins, stride, fields, fstride);
    return hipGetLastError();
}

__global__ void k_bump(int32_t* __restrict__ t_base, int d)
{
    if (threadIdx.x == 0) *t_base += d;
}

hipError_t launch_bump(int32_t* t_base, int d, hipStream_t st)
{
    hipLaunchKernelGGL(k_bump, dim3(1), dim3(64), 0, st, t_base, d);
    return hipGetLastError();
}

hipError_t launch_end(RepState* rs, int R, const int64_t* acc, int nslots, int T, int until_conv, int64_t n,
                      CallStats* cs, hipStream_t st, bool absolute)
{
    const unsigned threads = nslots <= 64 ? 64 : 256;
    hipLaunchKernelGGL(k_end, dim3(R), dim3(threads), 0, st, rs, acc, nslots, T, until_conv, n, cs,
                       absolute ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_any_active(const RepState* rs, int R, int T, uint32_t* flag, hipStream_t st)
{
    hipLaunchKernelGGL(k_any_active, dim3(grid1(R, 256, 1u << 30)), dim3(256), 0, st, rs, R, T, flag);
    return hipGetLastError();
}

hipError_t launch_philox_word0(const uint32_t* ctr, uint32_t* out, int64_t count, uint64_t seed, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_philox_word0, dim3(grid1((uint64_t)count, 256, 8192)), dim3(256), 0, st, ctr, out, count,
                       seed);
    return hipGetLastError();
}

hipError_t launch_best(const RepState* rs, const int64_t* rep_base, const int32_t* restarts, int ninst,
                       int64_t* Eb, int32_t* rb, hipStream_t st)
{
    hipLaunchKernelGGL(k_best, dim3(grid1((uint64_t)ninst * 64, 256, 1u << 30)), dim3(256), 0, st, rs, rep_base,
                       restarts, ninst, Eb, rb);
    return hipGetLastError();
}

}  // namespace sg
