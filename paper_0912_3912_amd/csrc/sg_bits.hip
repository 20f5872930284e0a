// sg_bits.hip -- the block schedule under GREEDY in bit-sliced form: one
// 32-bit LDS word holds spin i of 32 restarts of an instance (bit b set when
// restart b has s_i = -1), and one lane decides a row of the sliced layout for
// those 32 restarts with word operations.
//
// For spin i let W_i be the sum of |c| over its terms (field, couplings,
// hyper-couplings: Sec. II eq. (1), Sec. VI eq. (5)) and U_i the part of it
// carried by terms that s_i does not satisfy (c times the product of the
// term's spins negative).  Then s_i f_i = W_i - 2 U_i, and the local move
// lowers the energy (GREEDY) iff 2 U_i > W_i, i.e. U_i >= floor(W_i / 2) + 1.
// A term is unsatisfied in restart b iff the XOR of its spins' bits and of
// the coefficient's sign bit is 1, so U_i is a weighted sum of such masks.
// It is accumulated in an 8-bit bit-sliced counter started at
// 127 - floor(W_i / 2): bit 7 of the result is the flip mask.  Coefficients
// of magnitude at most 15 (4-bit weights) and W_i <= 255 keep the counter
// within 8 bits; the host routes other instances to the byte kernel.
//
// One wavefront per group of 32 restarts, NG groups per workgroup; each
// wavefront runs its own groups, without waiting for the others.  The 32
// restarts of a group sweep in lockstep; a restart that stops (converged, or
// out of sweeps) is masked out of its group, and a group whose restarts have
// all stopped writes its spins back and takes the next 32 restarts of the
// workgroup's range.  Flip counts per restart are kept as
// bit-sliced counters per lane and summed over lanes with ballots.  Energies
// are not tracked incrementally: a finished group computes them from its
// final spins and the instance's term list (the same integer the incremental
// sum would give).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sg_device.h"
#include "sg_launch.h"
#include "sg_layout.h"

namespace sg {

// One wavefront per group of 32 restarts: NG groups make a workgroup of 64 NG
// threads (measured on 4096 Chimera instances x 256 restarts, 8 groups:
// 3.57 ms with 512 threads, against 4.22 ms with 1024 threads, two
// wavefronts per group; smaller workgroups share a CU and hide each other's
// phase synchronisation).
template <int NG>
constexpr int bits_threads() { return 64 * NG; }

__device__ __forceinline__ int bits_coef(uint32_t w) { return (int)(int8_t)(w & 0xffu); }

// A += wt * u for a weight 0..15 and a mask u, on 8 bit-sliced words.
__device__ __forceinline__ void acc_add(uint32_t (&A)[8], uint32_t wt, uint32_t u)
{
    const uint32_t m0 = u & (0u - (wt & 1u));
    const uint32_t m1 = u & (0u - ((wt >> 1) & 1u));
    const uint32_t m2 = u & (0u - ((wt >> 2) & 1u));
    const uint32_t m3 = u & (0u - ((wt >> 3) & 1u));
    uint32_t c = A[0] & m0;
    A[0] ^= m0;
    {
        const uint32_t a = A[1];
        A[1] = a ^ m1 ^ c;
        c = (a & m1) | (c & (a ^ m1));
    }
    {
        const uint32_t a = A[2];
        A[2] = a ^ m2 ^ c;
        c = (a & m2) | (c & (a ^ m2));
    }
    {
        const uint32_t a = A[3];
        A[3] = a ^ m3 ^ c;
        c = (a & m3) | (c & (a ^ m3));
    }
#pragma unroll
    for (int b = 4; b < 8; ++b) {
        const uint32_t a = A[b];
        A[b] = a ^ c;
        c = a & c;
    }
}

// Four weighted masks at once: two 4-bit sums into 5 bits, their sum into 6
// bits, and that added into the 8-bit counter (fewer carry chains through the
// upper bits of A than four separate additions).
__device__ __forceinline__ void acc_add4(uint32_t (&A)[8], const uint32_t (&wt)[4], const uint32_t (&u)[4])
{
    uint32_t m[4][4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int p = 0; p < 4; ++p) m[t][p] = u[t] & (0u - ((wt[t] >> p) & 1u));
    uint32_t S[2][5];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const uint32_t* a = m[2 * h];
        const uint32_t* b = m[2 * h + 1];
        uint32_t c = a[0] & b[0];
        S[h][0] = a[0] ^ b[0];
#pragma unroll
        for (int p = 1; p < 4; ++p) {
            S[h][p] = a[p] ^ b[p] ^ c;
            c = (a[p] & b[p]) | (c & (a[p] ^ b[p]));
        }
        S[h][4] = c;
    }
    uint32_t T[6];
    {
        uint32_t c = S[0][0] & S[1][0];
        T[0] = S[0][0] ^ S[1][0];
#pragma unroll
        for (int p = 1; p < 5; ++p) {
            T[p] = S[0][p] ^ S[1][p] ^ c;
            c = (S[0][p] & S[1][p]) | (c & (S[0][p] ^ S[1][p]));
        }
        T[5] = c;
    }
    uint32_t c = A[0] & T[0];
    A[0] ^= T[0];
#pragma unroll
    for (int p = 1; p < 6; ++p) {
        const uint32_t a = A[p];
        A[p] = a ^ T[p] ^ c;
        c = (a & T[p]) | (c & (a ^ T[p]));
    }
#pragma unroll
    for (int p = 6; p < 8; ++p) {
        const uint32_t a = A[p];
        A[p] = a ^ c;
        c = a & c;
    }
}

__device__ __forceinline__ uint32_t wave_or(uint32_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v |= __shfl_xor(v, off, 64);
    return v;
}

template <int NG>
__global__ __launch_bounds__(bits_threads<NG>()) void k_block_bits(const InstTab* __restrict__ tab,
                                                             const int32_t* __restrict__ ctab,
                                                             const BlockItem* __restrict__ items,
                                                             RepState* __restrict__ rs, CallStats* __restrict__ cs,
                                                             int T, int until_conv)
{
    constexpr int kBitsThreads = bits_threads<NG>(), kBitsWaves = kBitsThreads / 64;
    constexpr int WPG = kBitsWaves / NG;  // wavefronts per group of 32 restarts
    static_assert(WPG == 1, "one wavefront per group");
    extern __shared__ uint64_t lds64[];
    const BlockItem it = items[blockIdx.x];
    const InstTab& Q = tab[it.inst];
    const InstDev& I = Q.I;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = wave % NG, wk = wave / NG;  // the wavefront's group, its index within the group
    const int n = I.n;
    const int r_end = it.r0 + it.nr;
    const int ew = Q.nbr_words, tw = Q.tri_words, nsl = I.nslices, C = Q.C;

    // LDS: couplings | triple words a | triple words b | slices | h | flip offsets | colour table |
    // spin words [NG][n] (group-major: a wavefront's neighbour reads spread over the banks) |
    // per-restart state [NG][32] x 3
    uint32_t* l_nbr = reinterpret_cast<uint32_t*>(lds64);
    uint32_t* l_ta = l_nbr + ew;
    uint32_t* l_tb = l_ta + tw;
    Slice* l_sl = reinterpret_cast<Slice*>(l_tb + tw + ((ew + 2 * tw) & 3 ? 4 - ((ew + 2 * tw) & 3) : 0));
    int8_t* l_h = reinterpret_cast<int8_t*>(l_sl + nsl);
    uint8_t* l_k = reinterpret_cast<uint8_t*>(l_h + ((n + 3) & ~3));
    int32_t* l_cs = reinterpret_cast<int32_t*>(l_k + ((n + 3) & ~3));
    uint32_t* l_sp = reinterpret_cast<uint32_t*>(l_cs + C + 1);
    int* r_t = reinterpret_cast<int*>(l_sp + (size_t)n * NG);  // sweeps of each restart in this call
    int* r_last = r_t + NG * 32;                                // 1 + its last sweep that flipped
    int* r_flips = r_last + NG * 32;                            // its flips in this call
    __shared__ int g_r0[NG], g_cnt[NG];                         // restarts [g_r0, g_r0 + g_cnt) in the group's bits
    __shared__ uint32_t g_act[NG], g_part[NG];                  // sweeping; taking part in the call
    __shared__ int next_r, kflush;
    __shared__ unsigned long long b_att, b_flips, b_smax, b_unconv;

    for (int k = tid; k < ew; k += kBitsThreads) l_nbr[k] = I.nbr[k];
    if (I.has_tri)
        for (int k = tid; k < tw; k += kBitsThreads) {
            l_ta[k] = I.ta[k];
            l_tb[k] = I.tb[k];
        }
    for (int k = tid; k < nsl; k += kBitsThreads) l_sl[k] = I.slices[k];
    for (int k = tid; k < n; k += kBitsThreads) l_h[k] = I.h[k];
    for (int k = tid; k <= C; k += kBitsThreads) l_cs[k] = ctab[Q.ctab_off + k];
    if (tid == 0) {
        next_r = it.r0;
        b_att = b_flips = b_smax = b_unconv = 0;
    }
    if (tid < NG) {
        g_cnt[tid] = 0;
        g_act[tid] = g_part[tid] = 0u;
    }
    __syncthreads();
    // flip offsets 127 - floor(W_i / 2); rows a lane decides per sweep (bounds the counters)
    for (int sl = wave; sl < nsl; sl += kBitsWaves) {
        const Slice S = l_sl[sl];
        if (lane < S.rows) {
            const int i = (int)S.row0 + lane;
            int W = abs((int)l_h[i]);
            for (int k = 0; k < S.ew; ++k) W += abs(bits_coef(l_nbr[S.ebase + k * kSlice + lane]));
            for (int k = 0; k < S.tw; ++k) W += abs(bits_coef(l_ta[S.tbase + k * kSlice + lane]));
            l_k[i] = (uint8_t)(127 - W / 2);
        }
    }
    if (tid == 0) {
        int rows = 0;
        for (int c = 0; c < C; ++c) rows += (l_cs[c + 1] - l_cs[c] + WPG - 1) / WPG;
        kflush = max(1, 255 / max(1, rows));  // sweeps between counter flushes
    }

    // next group of up to 32 restarts with at least one not frozen (the group's wavefront)
    auto fetch = [&]() {
        for (;;) {
            int r = 0;
            if (lane == 0) r = atomicAdd(&next_r, 32);
            r = __shfl(r, 0, 64);
            if (r >= r_end) {
                if (lane == 0) {
                    g_cnt[g] = 0;
                    g_act[g] = g_part[g] = 0u;
                }
                return false;
            }
            const int cnt = min(32, r_end - r);
            const bool live = lane < cnt && !rs[Q.rep_base + r + lane].converged;
            const uint32_t act = (uint32_t)__ballot(live);
            if (!act) continue;
            if (lane < 32) {
                r_t[g * 32 + lane] = 0;
                r_last[g * 32 + lane] = 0;
                r_flips[g * 32 + lane] = 0;
            }
            if (lane == 0) {
                g_r0[g] = r;
                g_cnt[g] = cnt;
                g_act[g] = g_part[g] = act;
            }
            return true;
        }
    };
    // spins of group g between global bytes and LDS words (its WPG
    // wavefronts): lane b + 32 h moves 16 consecutive spins of restart b, rows
    // [16 (2 q + h), +16) for chunk pair q, with one 16-byte access, and 16
    // ballots turn the bytes of 64 lanes into 32 spin words.  Rows past n in a
    // chunk stay within the replica's padded spin row and are not stored.
    auto load_group = [&]() {
        const int r0 = g_r0[g], cnt = g_cnt[g];
        const int b = lane & 31, hh = lane >> 5;
        for (int q = wk; q * 32 < n; q += WPG) {
            const int i0 = q * 32 + hh * 16;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (b < cnt && i0 < n)
                v = *reinterpret_cast<const uint4*>(Q.spins + (int64_t)(r0 + b) * Q.spin_stride + i0);
            const uint32_t wv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const uint64_t m = __ballot((wv[r >> 2] >> (8 * (r & 3) + 7)) & 1u);
                const int ia = q * 32 + r, ib = q * 32 + 16 + r;
                if (lane == r && ia < n) l_sp[g * n + ia] = (uint32_t)m;
                if (lane == 32 + r && ib < n) l_sp[g * n + ib] = (uint32_t)(m >> 32);
            }
        }
    };
    auto store_group = [&]() {
        const int r0 = g_r0[g], cnt = g_cnt[g];
        const int b = lane & 31, hh = lane >> 5;
        for (int q = wk; q * 32 < n; q += WPG) {
            const int i0 = q * 32 + hh * 16;
            if (b >= cnt || i0 >= n) continue;
            uint32_t wv[4] = {0u, 0u, 0u, 0u};
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int i = i0 + r;
                const uint32_t bit = i < n ? (l_sp[g * n + i] >> b) & 1u : 0u;
                wv[r >> 2] |= (bit ? 0xFFu : 0x01u) << (8 * (r & 3));
            }
            int8_t* dst = Q.spins + (int64_t)(r0 + b) * Q.spin_stride + i0;
            if (i0 + 16 <= n) {
                *reinterpret_cast<uint4*>(dst) = make_uint4(wv[0], wv[1], wv[2], wv[3]);
            } else {
                for (int r = 0; r < n - i0; ++r) dst[r] = (int8_t)((wv[r >> 2] >> (8 * (r & 3))) & 0xFFu);
            }
        }
    };

    // Energies of the group's 32 restarts from their final spins (Sec. II
    // eq. (1), Sec. VI eq. (5)): E = -sum c prod s = 2 V - W, with W = sum |c|
    // over the instance's terms and V the |c|-weighted count of unsatisfied
    // terms.  The lanes split the term list; each keeps an 8-bit bit-sliced
    // count (at most 16 terms of weight <= 15) that it folds into a 20-bit one
    // (sum |c| <= 2048 * 255 < 2^20 for the instances this kernel takes), and
    // ballots sum the lanes' counts per restart.  Lane b < 32 returns the
    // energy of restart b.
    const uint32_t* ET = Q.eterm;
    const int n_eh = Q.n_eh, n_ee = Q.n_ee, n_et = Q.n_et;
    auto group_energy = [&]() -> long long {
        const uint32_t* spg = l_sp + g * n;
        constexpr int kBW = 20;
        uint32_t A[8] = {0, 0, 0, 0, 0, 0, 0, 0}, B[kBW];
#pragma unroll
        for (int p = 0; p < kBW; ++p) B[p] = 0u;
        int wsum = 0, pending = 0;
        auto fold = [&]() {  // B += A, A = 0
            uint32_t c = 0;
#pragma unroll
            for (int p = 0; p < kBW; ++p) {
                const uint32_t a = p < 8 ? A[p] : 0u, bb = B[p];
                B[p] = bb ^ a ^ c;
                c = (bb & a) | (c & (bb ^ a));
            }
#pragma unroll
            for (int p = 0; p < 8; ++p) A[p] = 0u;
            pending = 0;
        };
        auto term = [&](uint32_t w, uint32_t parity) {
            const int cf = bits_coef(w >> 22);
            wsum += abs(cf);
            acc_add(A, (uint32_t)abs(cf), parity ^ (cf < 0 ? ~0u : 0u));
            if (++pending == 16) fold();
        };
        for (int t = lane; t < n_eh; t += 64) {
            const uint32_t w = ET[t];
            term(w, spg[w & 0x7FFu]);
        }
        for (int t = lane; t < n_ee; t += 64) {
            const uint32_t w = ET[n_eh + t];
            term(w, spg[w & 0x7FFu] ^ spg[(w >> 11) & 0x7FFu]);
        }
        for (int t = lane; t < n_et; t += 64) {
            const uint32_t w = ET[n_eh + n_ee + 2 * t], b = ET[n_eh + n_ee + 2 * t + 1];
            term(w, spg[w & 0x7FFu] ^ spg[(w >> 11) & 0x7FFu] ^ spg[b]);
        }
        fold();
        long long V = 0;
#pragma unroll
        for (int p = 0; p < kBW; ++p) {
            if (__ballot(B[p] != 0u) == 0) continue;
            for (int b = 0; b < 32; ++b) {
                const long long v = (long long)__popcll(__ballot((B[p] >> b) & 1u)) << p;
                if (lane == b) V += v;
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) wsum += __shfl_xor(wsum, off, 64);
        return 2 * V - (long long)wsum;
    };

    // Each wavefront runs its own group (one wavefront per group): it sweeps,
    // keeps its restarts' counters, finishes the group and takes the next
    // restarts without waiting for the other groups of the workgroup.  Its
    // LDS writes and later reads by other lanes of the same wavefront are
    // ordered by wavefront fences (LDS operations of a wavefront complete in
    // order; the fences keep the compiler from moving them).
    auto wave_sync = [] {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    __syncthreads();  // flip offsets and kflush are read by every wavefront
    bool have = fetch();
    wave_sync();
    if (have) load_group();
    wave_sync();

    uint32_t cnt8[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // this lane's flips per restart of its group, bit-sliced
    int since = 0;                                 // sweeps since the counters were last flushed
    uint32_t act = have ? g_act[g] : 0u;
    while (have) {
        uint32_t any = 0;
        for (int c = 0; c < C; ++c) {
            for (int sl = l_cs[c]; sl < l_cs[c + 1]; ++sl) {
                const Slice S = l_sl[sl];
                if (lane < S.rows) {
                    const int i = (int)S.row0 + lane;
                    uint32_t* sp = l_sp + g * n;
                    const uint32_t xi = sp[i];
                    const uint32_t K = l_k[i];
                    uint32_t A[8];
#pragma unroll
                    for (int b = 0; b < 8; ++b) A[b] = 0u - ((K >> b) & 1u);
                    {
                        const int h = l_h[i];
                        acc_add(A, (uint32_t)abs(h), xi ^ (h < 0 ? ~0u : 0u));
                    }
                    const uint32_t* pw = l_nbr + S.ebase + lane;
                    // four couplings at a time: their loads are issued together
                    int k = 0;
                    for (; k + 4 <= S.ew; k += 4) {
                        uint32_t w[4], xj[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) w[u] = pw[(k + u) * kSlice];
#pragma unroll
                        for (int u = 0; u < 4; ++u) xj[u] = sp[w[u] >> 8];
                        uint32_t wt[4], um[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int cj = bits_coef(w[u]);
                            wt[u] = (uint32_t)abs(cj);
                            um[u] = xi ^ xj[u] ^ (cj < 0 ? ~0u : 0u);
                        }
                        acc_add4(A, wt, um);
                    }
                    for (; k < S.ew; ++k) {
                        const uint32_t w = pw[k * kSlice];
                        const int cj = bits_coef(w);
                        acc_add(A, (uint32_t)abs(cj), xi ^ sp[w >> 8] ^ (cj < 0 ? ~0u : 0u));
                    }
                    if (I.has_tri) {
                        const uint32_t* pa = l_ta + S.tbase + lane;
                        const uint32_t* pb = l_tb + S.tbase + lane;
                        for (int k = 0; k < S.tw; ++k) {
                            const uint32_t wa = pa[k * kSlice];
                            const int ck = bits_coef(wa);
                            acc_add(A, (uint32_t)abs(ck),
                                    xi ^ sp[wa >> 8] ^ sp[pb[k * kSlice]] ^ (ck < 0 ? ~0u : 0u));
                        }
                    }
                    const uint32_t F = A[7] & act;
                    if (F) {
                        sp[i] = xi ^ F;
                        any |= F;
                        uint32_t carry = F;
#pragma unroll
                        for (int b = 0; b < 8; ++b) {
                            const uint32_t t = cnt8[b] & carry;
                            cnt8[b] ^= carry;
                            carry = t;
                        }
                    }
                }
            }
            wave_sync();
        }
        any = wave_or(any);
        // per-restart bookkeeping of the sweep
        bool done = false;
        if (lane < 32 && ((act >> lane) & 1u)) {
            const int t = ++r_t[g * 32 + lane];
            const bool flipped = (any >> lane) & 1u;
            if (flipped) r_last[g * 32 + lane] = t;
            done = (until_conv && !flipped) || t >= T;
        }
        act &= ~(uint32_t)__ballot(done);
        const bool fin = act == 0u;
        if (fin || ++since >= kflush) {
            // flip counters: per restart b, sum over lanes of each counter bit
            since = 0;
            int mine = 0;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (__ballot(cnt8[k] != 0u) == 0) continue;
                for (int b = 0; b < 32; ++b) {
                    const int v = (int)__popcll(__ballot((cnt8[k] >> b) & 1u)) << k;
                    if (lane == b) mine += v;
                }
                cnt8[k] = 0u;
            }
            if (lane < 32) r_flips[g * 32 + lane] += mine;
        }
        if (fin) {
            store_group();
            const long long Eg = group_energy();
            if (lane < 32 && ((g_part[g] >> lane) & 1u)) {
                const int t = r_t[g * 32 + lane], last = r_last[g * 32 + lane], nf = r_flips[g * 32 + lane];
                RepState* st = rs + Q.rep_base + g_r0[g] + lane;
                st->E = Eg;
                st->flips += nf;
                st->sweeps += t;
                st->lastflip = last;
                const bool conv = until_conv && last < t;
                if (conv) st->converged = 1;
                atomicAdd(&b_att, (unsigned long long)t * (unsigned long long)n);
                atomicAdd(&b_flips, (unsigned long long)nf);
                atomicMax(&b_smax, (unsigned long long)t);
                if (until_conv && !conv) atomicAdd(&b_unconv, 1ull);
            }
            wave_sync();
            have = fetch();
            wave_sync();
            if (have) load_group();
            wave_sync();
            act = have ? g_act[g] : 0u;
        }
    }
    __syncthreads();
    if (tid == 0) {
        if (b_att) atomicAdd(&cs->attempts, b_att);
        if (b_flips) atomicAdd(&cs->flips, b_flips);
        atomicMax(&cs->sweeps_max, b_smax);
        if (b_unconv) atomicAdd(&cs->unconverged, b_unconv);
    }
}

size_t block_bits_lds_bytes(int n, int nbr_words, int tri_words, int nslices, int C, int NG)
{
    size_t b = (size_t)nbr_words * 4 + (size_t)tri_words * 8;
    b = (b + 15) / 16 * 16;
    b += (size_t)nslices * sizeof(Slice);
    b += (size_t)((n + 3) & ~3) * 2;
    b += (size_t)(C + 1) * 4;
    b += (size_t)n * NG * 4;
    b += (size_t)NG * 32 * 4 * 3;
    return (b + 15) / 16 * 16;
}

template <int NG>
static hipError_t launch_bits_ng(const InstTab* tab, const int32_t* ctab, const BlockItem* items, int n_items,
                                 size_t lds, RepState* rs, CallStats* cs, int T, int until_conv, hipStream_t st)
{
    hipError_t e = hipFuncSetAttribute((const void*)k_block_bits<NG>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_block_bits<NG>, dim3(n_items), dim3(bits_threads<NG>()), lds, st, tab, ctab, items, rs, cs,
                       T, until_conv);
    return hipGetLastError();
}

hipError_t launch_block_bits(const InstTab* tab, const int32_t* ctab, const BlockItem* items, int n_items, size_t lds,
                             RepState* rs, CallStats* cs, int NG, int T, int until_conv, hipStream_t st)
{
    if (n_items <= 0) return hipSuccess;
    switch (NG) {
    case 2: return launch_bits_ng<2>(tab, ctab, items, n_items, lds, rs, cs, T, until_conv, st);
    case 4: return launch_bits_ng<4>(tab, ctab, items, n_items, lds, rs, cs, T, until_conv, st);
    case 8: return launch_bits_ng<8>(tab, ctab, items, n_items, lds, rs, cs, T, until_conv, st);
    case 16: return launch_bits_ng<16>(tab, ctab, items, n_items, lds, rs, cs, T, until_conv, st);
    default: return hipErrorInvalidValue;
    }
}

int block_bits_max_blocks(size_t lds, int NG)
{
    const void* kern = NG == 2 ? (const void*)k_block_bits<2>
                       : NG == 4 ? (const void*)k_block_bits<4>
                       : NG == 8 ? (const void*)k_block_bits<8>
                                 : (const void*)k_block_bits<16>;
    int per_cu = 0, dev = 0, cus = 0;
    if (hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * NG, lds) != hipSuccess ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return per_cu * cus;
}

}  // namespace sg
