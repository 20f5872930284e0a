// sg_fm.hip -- the paper's pass-based local search with hill-climbing
// (Sec. IV, Fig. 3), one wavefront per replica.
//
// A pass starts from the replica's state SP* and its tracked energy.  All
// gains g_i = -dE_i = -2 s_i f_i are evaluated; then, n times, the unlocked
// spin of largest gain (lowest external index among equal gains) is moved even
// when its gain is negative, the gains of its coupling and hyper-coupling
// partners are updated (a flip of s_i changes f_j by -2 J_ij s_i and
// f_a by -2 K s_i s_b), and the spin is locked; whenever the energy is
// strictly below the lowest seen in the pass, the prefix length is
// remembered.  At the end of the pass the moves after the best prefix are
// undone, so the best state seen becomes SP*.  Under until_converged the
// search stops after the first pass that does not lower the energy of SP*
// (that pass counts).  Counters: sweeps += passes, flips += moves kept,
// attempts = passes x n.
//
// Layout: the wavefront keeps the replica's gains (int32), spins (int8), the
// move list, and two index tables (internal index -> slice, -> external
// index) in its own LDS slice; couplings and hyper-couplings stay in the
// sliced layout in device memory (read through the cache, one word per lane
// per partner).  Lane l owns the internal indices l, l + 64, ...; it caches
// the best key of its unlocked spins, key = (gain + 2^30) << 32 | ~ext, and
// rescans its spins only when one of their gains changed or one was locked.
// The move is the wave-wide maximum key.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "sg_device.h"
#include <type_traits>
#include "sg_launch.h"
#include "sg_layout.h"

namespace sg {

constexpr int kFmThreads = 1024;
constexpr int kFmWaves = kFmThreads / 64;
constexpr int kFmGainBias = 1 << 30;

__host__ __device__ inline size_t fm_wave_bytes(int nmax)
{
    const size_t n4 = ((size_t)nmax + 3) & ~(size_t)3;
    return 4 * n4 + n4 + 2 * n4 + 2 * n4 + 2 * n4 + 16;  // gain, spin, move, slice, ext, dirty mask
}

__device__ __forceinline__ uint64_t fm_key(int gain, int ext)
{
    return ((uint64_t)(uint32_t)(gain + kFmGainBias) << 32) | (uint32_t)(0xFFFFFFFFu - (uint32_t)ext);
}

// One step of a wave-wide maximum through DPP lane permutations (no LDS
// traffic): lanes enabled by ROWS take the larger of their value and the
// permuted one; the others keep theirs.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint64_t dpp_max_step(uint64_t v)
{
    const int lo = (int)(uint32_t)v, hi = (int)(uint32_t)(v >> 32);
    const uint32_t lo2 = (uint32_t)__builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWS, 0xF, false);
    const uint32_t hi2 = (uint32_t)__builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWS, 0xF, false);
    const uint64_t w = ((uint64_t)hi2 << 32) | lo2;
    return w > v ? w : v;
}

// Maximum over the 64 lanes (every lane active): within quads, half-rows and
// rows by permutations, then across the four rows by the row broadcasts; lane
// 63 ends with the maximum, which is read back as a uniform value.
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v)
{
    v = dpp_max_step<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
    v = dpp_max_step<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
    v = dpp_max_step<0x141, 0xF>(v);  // row_half_mirror
    v = dpp_max_step<0x140, 0xF>(v);  // row_mirror
    v = dpp_max_step<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    v = dpp_max_step<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63);
    return ((uint64_t)hi << 32) | lo;
}

// The same in 32 bits, for instances whose gains satisfy |g| < 2^19 (the
// host checks 2 max_i sum|c| < 2^19) and whose external indices are below
// 4096: key = (g + 2^19) << 12 | (4095 - ext), ordered as the 64-bit key.
constexpr int kFmGainBias32 = 1 << 19;

__device__ __forceinline__ uint32_t fm_key32(int gain, int ext)
{
    return ((uint32_t)(gain + kFmGainBias32) << 12) | (uint32_t)(4095 - ext);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_max_step32(uint32_t v)
{
    const uint32_t w = (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, CTRL, ROWS, 0xF, false);
    return w > v ? w : v;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v)
{
    v = dpp_max_step32<0xB1, 0xF>(v);
    v = dpp_max_step32<0x4E, 0xF>(v);
    v = dpp_max_step32<0x141, 0xF>(v);
    v = dpp_max_step32<0x140, 0xF>(v);
    v = dpp_max_step32<0x142, 0xA>(v);
    v = dpp_max_step32<0x143, 0xC>(v);
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

__device__ __forceinline__ void wave_lds_order()
{
    // LDS operations of one wavefront complete in issue order; this keeps the
    // compiler from moving them across the point
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <bool TRI, bool K32>
__global__ __launch_bounds__(kFmThreads) void k_fm(const InstTab* __restrict__ tab, const int32_t* __restrict__ ctab,
                                                   const QueueItem* __restrict__ items, int nitems, int nmax,
                                                   int waves_per_block, RepState* __restrict__ rs,
                                                   CallStats* __restrict__ cs, uint32_t* __restrict__ err,
                                                   int max_passes, int until_conv, int stage_cap)
{
    extern __shared__ uint8_t fm_lds[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int item = blockIdx.x * waves_per_block + wave;
    long long att = 0, kept_all = 0;
    long long passes_done = 0;
    int unconv = 0;
    // When every wavefront of the block works on one instance (items are
    // instance-major), the block stages that instance's slices, coupling and
    // hyper-coupling words in LDS, so the partner reads of every move stay
    // on chip.
    const int first = blockIdx.x * waves_per_block;
    const int last = min(nitems, first + waves_per_block) - 1;
    const int inst0 = items[first].inst;
    const InstTab& Q0 = tab[inst0];
    const size_t stage_bytes = (size_t)Q0.I.nslices * sizeof(Slice) + (size_t)Q0.nbr_words * 4 +
                               (TRI ? (size_t)Q0.tri_words * 8 : 0);
    const bool staged = items[last].inst == inst0 && stage_bytes <= (size_t)stage_cap;
    InstDev IS = Q0.I;
    if (staged) {
        uint8_t* sbase = fm_lds + (size_t)waves_per_block * fm_wave_bytes(nmax);
        Slice* sl = reinterpret_cast<Slice*>(sbase);
        uint32_t* nb = reinterpret_cast<uint32_t*>(sl + Q0.I.nslices);
        uint32_t* ta = nb + Q0.nbr_words;
        uint32_t* tb = ta + (TRI ? Q0.tri_words : 0);
        for (int k = threadIdx.x; k < Q0.I.nslices; k += blockDim.x) sl[k] = Q0.I.slices[k];
        for (int k = threadIdx.x; k < Q0.nbr_words; k += blockDim.x) nb[k] = Q0.I.nbr[k];
        if (TRI)
            for (int k = threadIdx.x; k < Q0.tri_words; k += blockDim.x) {
                ta[k] = Q0.I.ta[k];
                tb[k] = Q0.I.tb[k];
            }
        IS.slices = sl;
        IS.nbr = nb;
        IS.ta = ta;
        IS.tb = tb;
    }
    __syncthreads();
    // The item body is instantiated once for the staged instance and once
    // for one read from global memory, so that in the first every slice and
    // coupling read is known to be an LDS access (a pointer that may be
    // either compiles to slower generic loads).
    auto body = [&](auto staged_tag, const InstDev I, const QueueItem it, const InstTab& Q) {
        (void)staged_tag;
        const int n = I.n;
        RepState* st = rs + Q.rep_base + it.r;
        if (!st->converged) {
            const size_t n4 = ((size_t)nmax + 3) & ~(size_t)3;
            uint8_t* base = fm_lds + (size_t)wave * fm_wave_bytes(nmax);
            int* gain = reinterpret_cast<int*>(base);
            int8_t* spin = reinterpret_cast<int8_t*>(base + 4 * n4);
            uint16_t* moves = reinterpret_cast<uint16_t*>(base + 5 * n4);
            uint16_t* slice_of = reinterpret_cast<uint16_t*>(base + 7 * n4);
            uint16_t* ext = reinterpret_cast<uint16_t*>(base + 9 * n4);
            uint32_t* dirty = reinterpret_cast<uint32_t*>(base + 11 * n4);
            int8_t* gs = Q.spins + Q.spin_stride * it.r;
            const int G = (n + 63) >> 6;
            // index tables and spins
            for (int c = 0; c < Q.C; ++c) {
                const int s0 = ctab[Q.ctab_off + c], s1 = ctab[Q.ctab_off + c + 1];
                for (int sl = s0; sl < s1; ++sl) {
                    const Slice S = I.slices[sl];
                    if (lane < S.rows) slice_of[S.row0 + lane] = (uint16_t)sl;
                }
            }
            for (int i = lane; i < n; i += 64) {
                ext[i] = (uint16_t)I.ext[i];
                spin[i] = gs[i];
            }
            if (lane < 2) dirty[lane] = 0u;
            wave_lds_order();
            long long Estar = st->E;
            int passes = 0;
            long long kept = 0;
            bool conv = false, bad = false;
            for (int pass = 0; pass < max_passes && !bad; ++pass) {
                // gains from the definition, and this lane's best unlocked key
                for (int i = lane; i < n; i += 64) {
                    const Slice S = I.slices[slice_of[i]];
                    const int l = i - (int)S.row0;
                    int f = I.h[i];
                    const uint32_t* p = I.nbr + S.ebase + l;
                    for (int k = 0; k < S.ew; ++k) {
                        const uint32_t w = p[k * kSlice];
                        f += (int)(int8_t)(w & 0xffu) * spin[w >> 8];
                    }
                    if (TRI) {
                        const uint32_t* pa = I.ta + S.tbase + l;
                        const uint32_t* pb = I.tb + S.tbase + l;
                        for (int k = 0; k < S.tw; ++k) {
                            const uint32_t wa = pa[k * kSlice];
                            f += (int)(int8_t)(wa & 0xffu) * spin[wa >> 8] * spin[pb[k * kSlice]];
                        }
                    }
                    gain[i] = -2 * spin[i] * f;
                }
                wave_lds_order();
                uint64_t locked = 0;
                using Key = std::conditional_t<K32, uint32_t, uint64_t>;
                auto make_key = [](int gn, int e) -> Key {
                    if constexpr (K32) return fm_key32(gn, e);
                    else return fm_key(gn, e);
                };
                // this lane's best unlocked key: its spins lane, lane + 64, ... in
                // groups of eight, every load of a group issued before any is used
                // (one LDS round trip per group instead of one per spin)
                auto scan = [&](uint64_t lk, Key& bk, int& bi) {
                    bk = 0;
                    bi = -1;
                    for (int k0 = 0; k0 < G; k0 += 8) {
                        Key kk[8];
#pragma unroll
                        for (int u = 0; u < 8; ++u) {
                            const int k = k0 + u;
                            const int ii = lane + 64 * k;
                            const bool ok = k < G && ii < n && !((lk >> (k & 63)) & 1ull);
                            const int is = ok ? ii : 0;
                            const int gv = gain[is];
                            const int ev = ext[is];
                            kk[u] = ok ? make_key(gv, ev) : Key(0);
                        }
#pragma unroll
                        for (int u = 0; u < 8; ++u)
                            if (kk[u] > bk) {
                                bk = kk[u];
                                bi = lane + 64 * (k0 + u);
                            }
                    }
                };
                Key best = 0;
                int besti = -1;
                scan(0ull, best, besti);
                long long E = Estar, Elow = Estar;
                int best_len = 0;
                for (int step = 0; step < n; ++step) {
                    Key top;
                    int g;
                    if constexpr (K32) {
                        top = wave_max_u32(best);
                        g = (int)(top >> 12) - kFmGainBias32;
                    } else {
                        top = wave_max_u64(best);
                        g = (int)(uint32_t)(top >> 32) - kFmGainBias;
                    }
                    // the move: the spin cached by the lane holding the maximum key
                    const uint64_t own = __ballot(best == top);
                    const int owner = (int)__builtin_ctzll(own);
                    const int i = __builtin_amdgcn_readlane(besti, owner);
                    if (i < 0) {  // a cached key without its spin: internal error, stop this replica
                        bad = true;
                        break;
                    }
                    const int s_old = spin[i];
                    const Slice S = I.slices[slice_of[i]];
                    const int l = i - (int)S.row0;
                    for (int k = lane; k < S.ew; k += 64) {
                        const uint32_t w = I.nbr[S.ebase + k * kSlice + l];
                        const int J = (int)(int8_t)(w & 0xffu);
                        if (J) {
                            const int j = (int)(w >> 8);
                            atomicAdd(gain + j, 4 * spin[j] * J * s_old);
                            atomicOr(dirty + ((j & 63) >> 5), 1u << (j & 31));
                        }
                    }
                    if (TRI) {
                        for (int k = lane; k < S.tw; k += 64) {
                            const uint32_t wa = I.ta[S.tbase + k * kSlice + l];
                            const int K = (int)(int8_t)(wa & 0xffu);
                            if (K) {
                                const int a = (int)(wa >> 8);
                                const int b = (int)I.tb[S.tbase + k * kSlice + l];
                                const int sa = spin[a], sb = spin[b];
                                atomicAdd(gain + a, 4 * sa * K * sb * s_old);
                                atomicAdd(gain + b, 4 * sb * K * sa * s_old);
                                atomicOr(dirty + ((a & 63) >> 5), 1u << (a & 31));
                                atomicOr(dirty + ((b & 63) >> 5), 1u << (b & 31));
                            }
                        }
                    }
                    wave_lds_order();
                    const uint32_t dm = dirty[lane >> 5];
                    bool rescan = (dm >> (lane & 31)) & 1u;
                    if (lane == owner) {
                        locked |= 1ull << (i >> 6);
                        spin[i] = (int8_t)-s_old;
                        moves[step] = (uint16_t)i;
                        rescan = true;
                    }
                    wave_lds_order();
                    if (lane < 2) dirty[lane] = 0u;
                    if (rescan) scan(locked, best, besti);
                    E -= g;
                    if (E < Elow) {
                        Elow = E;
                        best_len = step + 1;
                    }
                    wave_lds_order();
                }
                if (bad) break;
                // undo the moves after the best prefix
                for (int t = best_len + lane; t < n; t += 64) {
                    const int i = moves[t];
                    spin[i] = (int8_t)-spin[i];
                }
                wave_lds_order();
                ++passes;
                kept += best_len;
                const bool improved = Elow < Estar;
                Estar = Elow;
                if (until_conv && !improved) {
                    conv = true;
                    break;
                }
            }
            if (bad && lane == 0) atomicOr(err, 1u);
            for (int i = lane; i < n && !bad; i += 64) gs[i] = spin[i];
            if (lane == 0 && !bad) {
                st->E = Estar;
                st->sweeps += passes;
                st->flips += kept;
                if (conv) st->converged = 1;
            }
            att = (long long)passes * n;
            kept_all = kept;
            passes_done = passes;
            unconv = (until_conv && !conv) ? 1 : 0;
        }
    };
    if (wave < waves_per_block && item < nitems) {
        const QueueItem it = items[item];
        const InstTab& Q = tab[it.inst];
        if (staged)
            body(std::true_type{}, IS, it, Q);
        else
            body(std::false_type{}, Q.I, it, Q);
    }
    // call totals: one atomic per block
    __shared__ long long b_att, b_kept, b_passes;
    __shared__ int b_unconv;
    if (threadIdx.x == 0) {
        b_att = 0;
        b_kept = 0;
        b_passes = 0;
        b_unconv = 0;
    }
    __syncthreads();
    if (lane == 0 && (att || unconv)) {
        atomicAdd((unsigned long long*)&b_att, (unsigned long long)att);
        atomicAdd((unsigned long long*)&b_kept, (unsigned long long)kept_all);
        atomicMax((unsigned long long*)&b_passes, (unsigned long long)passes_done);
        atomicAdd(&b_unconv, unconv);
    }
    __syncthreads();
    if (threadIdx.x == 0 && (b_att || b_unconv)) {
        atomicAdd(&cs->attempts, (unsigned long long)b_att);
        atomicAdd(&cs->flips, (unsigned long long)b_kept);
        atomicMax(&cs->sweeps_max, (unsigned long long)b_passes);
        atomicAdd(&cs->unconverged, (unsigned long long)b_unconv);
    }
}

// The pass kernel for one instance in the wide form (any int32 coupling,
// field and hyper-coupling value with |h_i| + sum|J_ij| + sum|K| < 2^31 per
// spin): one wavefront per replica r in [0, R), waves_per_block wavefronts
// per workgroup.  The pass is that of k_fm.  Local fields fit int32, so each
// spin's half-gain v_i = -s_i f_i does too (the gain -dE_i is 2 v_i, up to
// 2^32 in magnitude); the wavefront keeps v in LDS and orders moves by the key
// (v + 2^31) << 32 | ~ext, larger gain first, then lower external index.  A
// flip of s_i changes a partner's half-gain by 2 J_ij s_i s_j, or by
// 2 K s_i s_a s_b for a hyper-coupling; the adds wrap modulo 2^32 on the way,
// and every half-gain they leave is again a value in range.
template <bool TRI>
__global__ __launch_bounds__(kFmThreads) void k_fm_wide(WideDev I, int8_t* __restrict__ spins, int64_t stride,
                                                        RepState* __restrict__ rs, int R, int nmax,
                                                        int waves_per_block, CallStats* __restrict__ cs,
                                                        uint32_t* __restrict__ err, int max_passes, int until_conv)
{
    extern __shared__ uint8_t fm_lds[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = blockIdx.x * waves_per_block + wave;
    long long att = 0, kept_all = 0, passes_done = 0;
    int unconv = 0;
    if (wave < waves_per_block && r < R && !rs[r].converged) {
        RepState* st = rs + r;
        const int n = I.n;
        const size_t n4 = ((size_t)nmax + 3) & ~(size_t)3;
        uint8_t* base = fm_lds + (size_t)wave * fm_wave_bytes(nmax);
        uint32_t* half = reinterpret_cast<uint32_t*>(base);  // v_i as two's complement
        int8_t* spin = reinterpret_cast<int8_t*>(base + 4 * n4);
        uint16_t* moves = reinterpret_cast<uint16_t*>(base + 5 * n4);
        uint16_t* slice_of = reinterpret_cast<uint16_t*>(base + 7 * n4);
        uint16_t* ext = reinterpret_cast<uint16_t*>(base + 9 * n4);
        uint32_t* dirty = reinterpret_cast<uint32_t*>(base + 11 * n4);
        int8_t* gs = spins + stride * r;
        const int G = (n + 63) >> 6;
        for (int sl = 0; sl < I.nslices; ++sl) {
            const WSlice S = I.slices[sl];
            if ((uint32_t)lane < S.rows) slice_of[S.row0 + lane] = (uint16_t)sl;
        }
        for (int i = lane; i < n; i += 64) {
            ext[i] = (uint16_t)I.ext[i];
            spin[i] = gs[i];
        }
        if (lane < 2) dirty[lane] = 0u;
        wave_lds_order();
        auto key_of = [](uint32_t v, int e) -> uint64_t {
            return ((uint64_t)(v ^ 0x80000000u) << 32) | (uint32_t)(0xFFFFFFFFu - (uint32_t)e);
        };
        // this lane's best unlocked key over its spins lane, lane + 64, ...
        auto scan = [&](uint64_t lk, uint64_t& bk, int& bi) {
            bk = 0;
            bi = -1;
            for (int k0 = 0; k0 < G; k0 += 8) {
                uint64_t kk[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int k = k0 + u, ii = lane + 64 * k;
                    const bool ok = k < G && ii < n && !((lk >> (k & 63)) & 1ull);
                    const int is = ok ? ii : 0;
                    kk[u] = ok ? key_of(half[is], ext[is]) : 0ull;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (kk[u] > bk) {
                        bk = kk[u];
                        bi = lane + 64 * (k0 + u);
                    }
            }
        };
        long long Estar = st->E, kept = 0;
        int passes = 0;
        bool conv = false, bad = false;
        for (int pass = 0; pass < max_passes && !bad; ++pass) {
            // half-gains from the definition (every partial sum of a local
            // field is bounded by the spin's limit, so int32 holds it)
            for (int i = lane; i < n; i += 64) {
                const WSlice S = I.slices[slice_of[i]];
                const uint32_t l = (uint32_t)i - S.row0;
                int32_t f = I.h[i];
                for (uint32_t k = 0; k < S.ew; ++k) {
                    const uint64_t o = S.ebase + (uint64_t)k * kSlice + l;
                    f += I.J[o] * spin[I.nbr[o]];
                }
                if (TRI)
                    for (uint32_t k = 0; k < S.tw; ++k) {
                        const uint64_t o = S.tbase + (uint64_t)k * kSlice + l;
                        f += I.K[o] * spin[I.ta[o]] * spin[I.tb[o]];
                    }
                half[i] = (uint32_t)(-spin[i] * f);
            }
            wave_lds_order();
            uint64_t locked = 0, best = 0;
            int besti = -1;
            scan(0ull, best, besti);
            long long E = Estar, Elow = Estar;
            int best_len = 0;
            for (int step = 0; step < n; ++step) {
                const uint64_t top = wave_max_u64(best);
                const int v = (int)((uint32_t)(top >> 32) ^ 0x80000000u);
                const uint64_t own = __ballot(best == top);
                const int owner = (int)__builtin_ctzll(own);
                const int i = __builtin_amdgcn_readlane(besti, owner);
                if (i < 0) {  // a cached key without its spin: internal error, stop this replica
                    bad = true;
                    break;
                }
                const int s_old = spin[i];
                const WSlice S = I.slices[slice_of[i]];
                const uint32_t l = (uint32_t)i - S.row0;
                for (uint32_t k = lane; k < S.ew; k += 64) {
                    const uint64_t o = S.ebase + (uint64_t)k * kSlice + l;
                    const int32_t J = I.J[o];
                    if (J) {
                        const uint32_t j = I.nbr[o];
                        atomicAdd(half + j, (uint32_t)J * (uint32_t)(2 * spin[j] * s_old));
                        atomicOr(dirty + ((j & 63u) >> 5), 1u << (j & 31u));
                    }
                }
                if (TRI)
                    for (uint32_t k = lane; k < S.tw; k += 64) {
                        const uint64_t o = S.tbase + (uint64_t)k * kSlice + l;
                        const int32_t K = I.K[o];
                        if (K) {
                            const uint32_t a = I.ta[o], b = I.tb[o];
                            const uint32_t d = (uint32_t)K * (uint32_t)(2 * spin[a] * spin[b] * s_old);
                            atomicAdd(half + a, d);
                            atomicAdd(half + b, d);
                            atomicOr(dirty + ((a & 63u) >> 5), 1u << (a & 31u));
                            atomicOr(dirty + ((b & 63u) >> 5), 1u << (b & 31u));
                        }
                    }
                wave_lds_order();
                const uint32_t dm = dirty[lane >> 5];
                bool rescan = (dm >> (lane & 31)) & 1u;
                if (lane == owner) {
                    locked |= 1ull << (i >> 6);
                    spin[i] = (int8_t)-s_old;
                    moves[step] = (uint16_t)i;
                    rescan = true;
                }
                wave_lds_order();
                if (lane < 2) dirty[lane] = 0u;
                if (rescan) scan(locked, best, besti);
                E -= 2LL * v;
                if (E < Elow) {
                    Elow = E;
                    best_len = step + 1;
                }
                wave_lds_order();
            }
            if (bad) break;
            // undo the moves after the best prefix
            for (int t = best_len + lane; t < n; t += 64) {
                const int i = moves[t];
                spin[i] = (int8_t)-spin[i];
            }
            wave_lds_order();
            ++passes;
            kept += best_len;
            const bool improved = Elow < Estar;
            Estar = Elow;
            if (until_conv && !improved) {
                conv = true;
                break;
            }
        }
        if (bad && lane == 0) atomicOr(err, 1u);
        for (int i = lane; i < n && !bad; i += 64) gs[i] = spin[i];
        if (lane == 0 && !bad) {
            st->E = Estar;
            st->sweeps += passes;
            st->flips += kept;
            if (conv) st->converged = 1;
        }
        att = (long long)passes * n;
        kept_all = kept;
        passes_done = passes;
        unconv = (until_conv && !conv) ? 1 : 0;
    }
    // call totals: one atomic per wavefront that ran a replica
    if (lane == 0 && (att || unconv)) {
        atomicAdd(&cs->attempts, (unsigned long long)att);
        atomicAdd(&cs->flips, (unsigned long long)kept_all);
        atomicMax(&cs->sweeps_max, (unsigned long long)passes_done);
        atomicAdd(&cs->unconverged, (unsigned long long)unconv);
    }
}

size_t fm_lds_bytes(int nmax, int waves) { return fm_wave_bytes(nmax) * (size_t)waves; }

template <bool TRI, bool K32>
static hipError_t launch_fm_t(const InstTab* tab, const int32_t* ctab, const QueueItem* items, int nitems, int nmax,
                              int waves, int stage_cap, RepState* rs, CallStats* cs, uint32_t* err, int max_passes,
                              int until_conv, hipStream_t st)
{
    const size_t lds = fm_lds_bytes(nmax, waves) + (size_t)stage_cap;
    hipError_t e = hipFuncSetAttribute((const void*)k_fm<TRI, K32>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    const int blocks = (nitems + waves - 1) / waves;
    hipLaunchKernelGGL((k_fm<TRI, K32>), dim3(blocks), dim3(waves * 64), lds, st, tab, ctab, items, nitems, nmax,
                       waves, rs, cs, err, max_passes, until_conv, stage_cap);
    return hipGetLastError();
}

template <bool TRI, bool K32>
static int fm_blocks_per_cu(int waves, size_t lds)
{
    const void* kern = (const void*)k_fm<TRI, K32>;
    int per_cu = 0;
    if (hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, waves * 64, lds) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return per_cu;
}

int fm_max_blocks_per_cu(int waves, size_t lds, bool tri, bool key32)
{
    if (tri) return key32 ? fm_blocks_per_cu<true, true>(waves, lds) : fm_blocks_per_cu<true, false>(waves, lds);
    return key32 ? fm_blocks_per_cu<false, true>(waves, lds) : fm_blocks_per_cu<false, false>(waves, lds);
}

hipError_t launch_fm_wide(const WideDev& I, int8_t* spins, int64_t stride, RepState* rs, int R, CallStats* cs,
                          uint32_t* err, int max_passes, int until_conv, hipStream_t st)
{
    if (R <= 0) return hipSuccess;
    if (I.n < 1 || I.n > 4096) return hipErrorInvalidValue;
    const size_t per = fm_wave_bytes(I.n);
    const int waves = (int)std::max<size_t>(1, std::min<size_t>(4, (size_t)(64 * 1024) / per));
    const size_t lds = per * (size_t)waves;
    const bool tri = I.has_tri != 0;
    const void* kern = tri ? (const void*)k_fm_wide<true> : (const void*)k_fm_wide<false>;
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const unsigned blocks = (unsigned)((R + waves - 1) / waves);
    if (tri)
        hipLaunchKernelGGL(k_fm_wide<true>, dim3(blocks), dim3(waves * 64), lds, st, I, spins, stride, rs, R, I.n,
                           waves, cs, err, max_passes, until_conv);
    else
        hipLaunchKernelGGL(k_fm_wide<false>, dim3(blocks), dim3(waves * 64), lds, st, I, spins, stride, rs, R, I.n,
                           waves, cs, err, max_passes, until_conv);
    return hipGetLastError();
}

hipError_t launch_fm(const InstTab* tab, const int32_t* ctab, const QueueItem* items, int nitems, int nmax, int waves,
                     int stage_cap, bool tri, bool key32, RepState* rs, CallStats* cs, uint32_t* err,
                     int max_passes, int until_conv, hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    if (waves < 1 || waves > kFmWaves || stage_cap < 0) return hipErrorInvalidValue;
    if (key32 && nmax > 4096) return hipErrorInvalidValue;
    if (tri)
        return key32 ? launch_fm_t<true, true>(tab, ctab, items, nitems, nmax, waves, stage_cap, rs, cs, err,
                                                max_passes, until_conv, st)
                     : launch_fm_t<true, false>(tab, ctab, items, nitems, nmax, waves, stage_cap, rs, cs, err,
                                                 max_passes, until_conv, st);
    return key32 ? launch_fm_t<false, true>(tab, ctab, items, nitems, nmax, waves, stage_cap, rs, cs, err, max_passes,
                                            until_conv, st)
                 : launch_fm_t<false, false>(tab, ctab, items, nitems, nmax, waves, stage_cap, rs, cs, err,
                                             max_passes, until_conv, st);
}

}  // namespace sg
