// sg_msc.hip -- multi-spin coded colour-ordered sweeps on periodic 2-D/3-D
// lattices whose couplings are all +-1 and whose fields satisfy |h| <= 2,
// LDS-resident tiles.
//
// Same tiling, halo, epoch and exchange protocol as k_lattice_tiles (a tile
// plus a halo of width k per workgroup, k colour phases between exchanges,
// bit-packed interior z-rows published as coherent 8-byte words that carry
// their epoch tag, bounded waits), but the box is held as bit-planes: every box
// z-row is split by colour into two 32-bit words (bit j of colour c's word
// is the site z = 2j + zo, zo = the row's offset for that colour), for the
// spin (bit set when s = -1), the sign of the +x, +y and +z bond (bit set
// when J = -1) and three field planes (h > 0, h < 0, |h| = 2).  One lane
// updates all sites of one colour of one row at once:
//
//   a bond (i, d) is unsatisfied when J s_i s_d = -1, i.e. when
//   bit(s_i) ^ bit(s_d) ^ bit(J < 0) = 1; with U = number of unsatisfied
//   bonds of i (a bit-sliced sum of 2D one-bit inputs) and g = s_i h_i,
//   s_i f_i = g + 2D - 2U, so dE_i = 2 s_i f_i = 2g + 4D - 4U
//   (the move cost of Sec. IV, the field of Sec. II eq. (1)).
//
// dE_i < 0 iff U >= D + 1 + (g == 2) - (g < 0); dE_i == 0 iff g is even and
// U equals that threshold minus one.  Both tests are bit-sliced compares of
// U against per-site thresholds selected by the g < 0 and g == 2 masks.
// Under GREEDY_TIE the dE == 0 sites of a wavefront's rows are compacted into
// the wavefront's own LDS segment and drawn from Philox by all of its lanes
// right after those rows (only this wavefront touches their words in this
// phase), so the draws run at full lane occupancy without a workgroup
// barrier.
//
// Energy: the phases count flips only.  After the last exchange (whose words
// then fill the whole box) each tile sums the exact energy of its interior:
// every interior site adds its +x, +y, +z bonds (+1 unsatisfied, -1
// satisfied) and -s h, so each bond and field of the lattice is counted once
// (Sec. II eq. (1)); the replica's energy is the sum over its tiles.
//
// Stopping rule (CONV, GREEDY only): after each sweep every tile adds one
// arrival and whether its interior flipped anything to that sweep's counter.
// Under GREEDY a sweep without a flip anywhere is a fixed point, so sweeps run
// after it change no spin: a tile keeps sweeping until it knows.  Once the
// counter of sweep s shows every tile arrived and none flipped, the tiles stop
// after exchange S - 1, S = e(s) + d + 2, where e(s) is the epoch holding the
// sweep's last phase and d the largest tile distance (Chebyshev, on the torus
// of tiles).  Every tile reads the counters after each exchange; a tile that
// finished exchange e has received words that depend on every tile within
// distance dd having finished exchange e - dd, so by exchange e(s) + d every
// tile has seen the completed counter and all stop after the same exchange.
// The replica's sweep count (the first sweep without a flip, plus one) is
// settled from the counters after the launch.
//
// Neighbours: the +-x and +-y neighbours of a colour-c site are the same bit
// of the other colour's word in the neighbouring rows (their offset is the
// same); its -z and +z neighbours are, in the same row's other-colour word,
// bits j-1 and j (zo = 0) or j and j+1 (zo = 1).  A -d bond is the +d bond of
// the -d neighbour, read from that neighbour's plane the same way.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "sg_device.h"
#include "sg_launch.h"
#include "sg_layout.h"

namespace sg {

constexpr int kMscThreads = 1024;
constexpr int kMscWaves = kMscThreads / 64;
constexpr int kExRows = 4;  // box rows per thread in the exchange (rows <= kExRows * kMscThreads)
constexpr int kWaveTieCap = 128;  // tie entries per wavefront segment (more are drawn in further rounds)

// plane indices (the +x plane exists for 3-D lattices only)
enum { kPlS = 0, kPlJY = 1, kPlJZ = 2, kPlHP = 3, kPlHN = 4, kPlHA = 5, kPlJX = 6 };

__host__ __device__ constexpr int msc_planes(int D) { return D == 3 ? 7 : 6; }

__device__ __forceinline__ int msc_jb(uint64_t rec, int k) { return (int)(int8_t)(rec >> (8 * k)); }

// bit i of x -> bit 2i (x < 2^16)
__device__ __forceinline__ uint32_t spread16(uint32_t x)
{
    x = (x | (x << 8)) & 0x00FF00FFu;
    x = (x | (x << 4)) & 0x0F0F0F0Fu;
    x = (x | (x << 2)) & 0x33333333u;
    x = (x | (x << 1)) & 0x55555555u;
    return x;
}
__device__ __forceinline__ uint64_t spread32(uint32_t x)
{
    return (uint64_t)spread16(x & 0xFFFFu) | ((uint64_t)spread16(x >> 16) << 32);
}
// bit 2i of x -> bit i
__device__ __forceinline__ uint32_t even16(uint32_t x)
{
    x &= 0x55555555u;
    x = (x | (x >> 1)) & 0x33333333u;
    x = (x | (x >> 2)) & 0x0F0F0F0Fu;
    x = (x | (x >> 4)) & 0x00FF00FFu;
    x = (x | (x >> 8)) & 0x0000FFFFu;
    return x;
}
__device__ __forceinline__ uint32_t even32(uint64_t v)
{
    return even16((uint32_t)v) | (even16((uint32_t)(v >> 32)) << 16);
}
// bits lo..hi (inclusive) set; empty when hi < lo; 0 <= lo <= 31
__device__ __forceinline__ uint32_t bit_range(int lo, int hi)
{
    if (hi < lo) return 0u;
    const uint32_t up = hi >= 31 ? 0xFFFFFFFFu : ((2u << hi) - 1u);
    return up & ~((1u << lo) - 1u);
}
__device__ __forceinline__ uint32_t low_bits(int n) { return n >= 32 ? 0xFFFFFFFFu : ((1u << n) - 1u); }

// full adder on bit-planes
__device__ __forceinline__ void fadd(uint32_t a, uint32_t b, uint32_t c, uint32_t& s, uint32_t& cy)
{
    const uint32_t t = a ^ b;
    s = t ^ c;
    cy = (t & c) | (~t & a);
}

// U >= t and U == t for U = (u2 u1 u0), 0 <= U <= 6
template <int t>
__device__ __forceinline__ uint32_t u_ge(uint32_t u0, uint32_t u1, uint32_t u2)
{
    static_assert(t >= 1 && t <= 6, "threshold");
    if constexpr (t == 1) return u2 | u1 | u0;
    else if constexpr (t == 2) return u2 | u1;
    else if constexpr (t == 3) return u2 | (u1 & u0);
    else if constexpr (t == 4) return u2;
    else if constexpr (t == 5) return u2 & (u1 | u0);
    else return u2 & u1;
}
template <int t>
__device__ __forceinline__ uint32_t u_eq(uint32_t u0, uint32_t u1, uint32_t u2)
{
    static_assert(t >= 0 && t <= 6, "value");
    return ((t & 4) ? u2 : ~u2) & ((t & 2) ? u1 : ~u1) & ((t & 1) ? u0 : ~u0);
}

template <int D, bool TIE, bool CONV>
__global__ __launch_bounds__(kMscThreads) void k_lattice_msc(LatticeDev Lt, TileGeom tg, int8_t* __restrict__ canon,
                                                             int64_t stride, uint64_t* __restrict__ G0,
                                                             uint64_t* __restrict__ G1, uint32_t* __restrict__ err, RepState* __restrict__ rs,
                                                             int64_t* __restrict__ acc, int nslots, int T,
                                                             uint64_t seed, uint64_t* __restrict__ scnt, int drift)
{
    static_assert(!(CONV && TIE), "the stopping rule runs on the tile kernel under GREEDY only");
    constexpr int NPL = msc_planes(D);
    constexpr int T0 = D + 1;  // flip threshold on U for g in {0, 1}
    extern __shared__ uint32_t lds32[];
    const int ntiles = tg.P[0] * tg.P[1] * tg.P[2];
    const int tile = blockIdx.x % ntiles;
    const int r = blockIdx.x / ntiles;
    // a replica frozen by an earlier call is not swept; all its tiles leave
    // together, and no other replica waits on them (exchanges are per replica)
    if (rs[r].converged) return;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int L0 = Lt.L[0], L1 = Lt.L[1], L2 = Lt.L[2];
    const int half = Lt.n / 2;
    const int k = tg.k;
    int tc[3];
    tc[0] = tile / (tg.P[1] * tg.P[2]);
    tc[1] = (tile / tg.P[2]) % tg.P[1];
    tc[2] = tile % tg.P[2];
    int X[3], hk[3], B[3], o[3], st[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int La = Lt.L[a];
        st[a] = (int)((int64_t)tc[a] * La / tg.P[a]);
        X[a] = (int)((int64_t)(tc[a] + 1) * La / tg.P[a]) - st[a];
        hk[a] = (D == 2 && a == 0) ? 0 : k;
        B[a] = X[a] + 2 * hk[a];
        o[a] = st[a] - hk[a];
    }
    // colour of box site (x, y, z) = (par0 + x + y + z) mod 2
    const int par0 = (((o[0] % 2) + (o[1] % 2) + (o[2] % 2) + Lt.c0) % 2 + 2) % 2;
    const int rows = B[0] * B[1];
    const int nrow_int = X[0] * X[1];
    const uint32_t mB1 = fdiv_magic((uint32_t)B[1]), mX1 = fdiv_magic((uint32_t)X[1]);
    auto tstart = [&](int a, int t) -> int { return (int)((int64_t)t * Lt.L[a] / tg.P[a]); };
    const int tzm = (tc[2] + tg.P[2] - 1) % tg.P[2], tzp = (tc[2] + 1) % tg.P[2];
    const int Xzm = tstart(2, tzm + 1) - tstart(2, tzm);
    // box row layout: RS words per row, word 2 * plane + colour; RS is odd, so
    // lanes on consecutive rows read distinct banks, and a row's words sit at
    // constant offsets from one address
    constexpr int RS = 2 * NPL + 1;
    auto pw = [&](int pl, int c, int row) -> uint32_t& { return lds32[row * RS + 2 * pl + c]; };
    // tie queue entries: (box row | z << 16 | interior << 22, global row index)
    uint2* tieq = reinterpret_cast<uint2*>(lds32 + ((RS * rows + 1) & ~1));
    __shared__ uint32_t mag_ay[64];
    int8_t* cs = canon + (int64_t)r * stride;
    const int rows_per_tile = ((L0 + tg.P[0] - 1) / tg.P[0]) * ((L1 + tg.P[1] - 1) / tg.P[1]);
    uint64_t* g0 = G0 + (int64_t)r * ntiles * rows_per_tile;
    uint64_t* g1 = G1 + (int64_t)r * ntiles * rows_per_tile;
    const uint32_t base = (uint32_t)rs[r].sweeps;
    auto gsite = [&](int x, int y, int z) -> int {
        return (wrapi(o[0] + x, L0) * L1 + wrapi(o[1] + y, L1)) * L2 + wrapi(o[2] + z, L2);
    };

    if (tid < 64) mag_ay[tid] = fdiv_magic((uint32_t)max(1, B[1] - 2 * (tid + 1)));
    // ---- bit-planes of the box: one wavefront per box row, lane = z
    for (int row = wave; row < rows; row += kMscWaves) {
        const int x = (int)fdiv((uint32_t)row, mB1);
        const int y = row - x * B[1];
        const int pr = (par0 + x + y) & 1;  // colour of the even-z sites
        const int z = lane;
        bool sneg = false, jx = false, jy = false, jz = false, hp = false, hn = false, ha = false;
        if (z < B[2]) {
            const int g = gsite(x, y, z);
            const uint64_t rc = Lt.rec[g];
            sneg = cs[((pr + z) & 1) * half + (g >> 1)] < 0;
            jx = msc_jb(rc, 0) < 0;
            jy = msc_jb(rc, 2) < 0;
            jz = msc_jb(rc, 4) < 0;
            const int hv = msc_jb(rc, 6);
            hp = hv > 0;
            hn = hv < 0;
            ha = hv == 2 || hv == -2;
        }
        const uint64_t m[7] = {__ballot(sneg), __ballot(jy), __ballot(jz), __ballot(hp),
                               __ballot(hn),   __ballot(ha), __ballot(jx)};
        if (lane < NPL) {
            uint64_t v = m[0];
#pragma unroll
            for (int pl = 1; pl < 7; ++pl)
                if (lane == pl) v = m[pl];
            pw(lane, pr, row) = even32(v);
            pw(lane, pr ^ 1, row) = even32(v >> 1);
        }
    }
    // where each of this thread's box rows (tid + kMscThreads * m) is read
    // from in the exchange buffers: the owning tile's first word plus the
    // row's index inside that tile (the same in every epoch, so the divisions
    // are done once per launch)
    int32_t exoff[kExRows];
#pragma unroll
    for (int m = 0; m < kExRows; ++m) {
        const int row = tid + m * kMscThreads;
        exoff[m] = 0;
        if (row >= rows) continue;
        const int x = (int)fdiv((uint32_t)row, mB1);
        const int y = row - x * B[1];
        const int gx = wrapi(o[0] + x, L0), gy = wrapi(o[1] + y, L1);
        const int tx = (int)(((int64_t)(gx + 1) * tg.P[0] - 1) / L0);
        const int ty = (int)(((int64_t)(gy + 1) * tg.P[1] - 1) / L1);
        const int sx = tstart(0, tx), sy = tstart(1, ty);
        const int X1t = tstart(1, ty + 1) - sy;
        const int wrow = (gx - sx) * X1t + (gy - sy);
        const int tb = (tx * tg.P[1] + ty) * tg.P[2];
        exoff[m] = tb * rows_per_tile + wrow;
    }
    __syncthreads();

    const int P_total = 2 * T;
    int nflip = 0;
    bool failed = false;
    // stopping rule: this replica's per-sweep counters, the next sweep to
    // read, and the epoch before which every tile of the replica stops
    uint64_t* const sc = CONV ? scnt + (int64_t)r * T : nullptr;
    __shared__ int s_next, s_stop;
    uint32_t fsw = 0;  // interior flips of this thread in the current sweep
    if (CONV && tid == 0) {
        s_next = 0;
        s_stop = 0x7FFFFFFF;
    }

    for (int e = 0; e * k < P_total; ++e) {
        const int nq = min(k, P_total - e * k);
        for (int q = 0; q < nq; ++q) {
            const int p = e * k + q;
            const int c = p & 1;
            const uint32_t sweep = base + (uint32_t)(p >> 1);
            const int ax = D == 3 ? B[0] - 2 * (q + 1) : 1;
            const int ay = B[1] - 2 * (q + 1);
            const int xlo = D == 3 ? q + 1 : 0, ylo = q + 1;
            const int nact = (ax > 0 && ay > 0) ? ax * ay : 0;
            const uint32_t may = mag_ay[q];
            // sites deeper than q along z, and the tile interior along z, per offset
            const uint32_t zm0 = bit_range((q + 2) >> 1, (B[2] - 2 - q) >> 1);
            const uint32_t zm1 = bit_range((q + 1) >> 1, (B[2] - 3 - q) >> 1);
            const uint32_t im0 = bit_range((hk[2] + 1) >> 1, (hk[2] + X[2] - 1) >> 1);
            const uint32_t im1 = bit_range(hk[2] >> 1, (hk[2] + X[2] - 2) >> 1);
            uint32_t* const Sc = lds32 + c;  // colour-c spin word of box row t: Sc[t * RS]
            // wave-uniform trip count: the tie queue is reserved once per wavefront
            for (int i0 = wave * 64; i0 < nact; i0 += kMscThreads) {
                const int i = i0 + lane;
                const bool act = i < nact;
                const int ii = act ? i : i0;
                const int qq = (int)fdiv((uint32_t)ii, may);
                const int x = xlo + qq, y = ylo + ii - qq * ay;
                const int row = x * B[1] + y;
                const int zo = (c - par0 - x - y) & 1;
                // this row's words of colour c and of the other colour
                uint32_t* const wc = lds32 + row * RS + c;
                const uint32_t* const wo = lds32 + row * RS + (c ^ 1);
                const uint32_t s = wc[2 * kPlS];
                const uint32_t on = wo[2 * kPlS];
                const uint32_t jzo = wo[2 * kPlJZ];
                const uint32_t szp = zo ? (on >> 1) : on;
                const uint32_t szm = zo ? on : (on << 1);
                const uint32_t jzm = zo ? jzo : (jzo << 1);
                const uint32_t a0 = s ^ wo[RS + 2 * kPlS] ^ wc[2 * kPlJY];
                const uint32_t a1 = s ^ wo[2 * kPlS - RS] ^ wo[2 * kPlJY - RS];
                const uint32_t a2 = s ^ szp ^ wc[2 * kPlJZ];
                const uint32_t a3 = s ^ szm ^ jzm;
                uint32_t u0, u1, u2;
                if constexpr (D == 3) {
                    const int BR = B[1] * RS;
                    const uint32_t a4 = s ^ wo[BR + 2 * kPlS] ^ wc[2 * kPlJX];
                    const uint32_t a5 = s ^ wo[2 * kPlS - BR] ^ wo[2 * kPlJX - BR];
                    uint32_t s1, c1, s2, c2;
                    fadd(a0, a1, a2, s1, c1);
                    fadd(a3, a4, a5, s2, c2);
                    u0 = s1 ^ s2;
                    fadd(c1, c2, s1 & s2, u1, u2);
                } else {
                    uint32_t s1, c1;
                    fadd(a0, a1, a2, s1, c1);
                    u0 = s1 ^ a3;
                    const uint32_t k0 = s1 & a3;
                    u1 = c1 ^ k0;
                    u2 = c1 & k0;
                }
                const uint32_t hp = wc[2 * kPlHP], hn = wc[2 * kPlHN], ha = wc[2 * kPlHA];
                const uint32_t gpos = (hp & ~s) | (hn & s);
                const uint32_t gneg = (hn & ~s) | (hp & s);
                const uint32_t gtwo = gpos & ha;  // g == +2
                const uint32_t gmid = ~(gneg | gtwo);
                const uint32_t M = act ? (zo ? zm1 : zm0) : 0u;
                const uint32_t flip = (gneg & u_ge<T0 - 1>(u0, u1, u2)) | (gtwo & u_ge<T0 + 1>(u0, u1, u2)) |
                                      (gmid & u_ge<T0>(u0, u1, u2));
                const uint32_t F = flip & M;
                const bool inner_row = x >= hk[0] && x < hk[0] + X[0] && y >= hk[1] && y < hk[1] + X[1];
                const uint32_t I = inner_row ? (zo ? im1 : im0) : 0u;
                const uint32_t FI = F & I;
                nflip += __popc(FI);
                if constexpr (CONV) fsw |= FI;
                const uint32_t ns = s ^ F;
                if constexpr (TIE) {
                    const uint32_t odd = (hp | hn) & ~ha;
                    const uint32_t tie = ~odd & ((gneg & u_eq<T0 - 2>(u0, u1, u2)) | (gtwo & u_eq<T0>(u0, u1, u2)) |
                                                 (gmid & u_eq<T0 - 1>(u0, u1, u2)));
                    const uint32_t Tm = tie & M;
                    if (ns != s) wc[2 * kPlS] = ns;
                    const int cnt = __popc(Tm);
                    if (__ballot(cnt != 0)) {
                        // exclusive prefix sum of the lanes' tie counts from one
                        // ballot per bit of the count (two bits unless some lane
                        // has more than three ties)
                        int below = 0, total = 0;
                        auto count_bit = [&](int b) {
                            const uint64_t m = __ballot((cnt >> b) & 1);
                            below += (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u))
                                     << b;
                            total += __popcll(m) << b;
                        };
                        count_bit(0);
                        count_bit(1);
                        if (__ballot(cnt > 3)) {
#pragma unroll
                            for (int b = 2; b < 6; ++b) count_bit(b);
                        }
                        uint2* seg = tieq + wave * kWaveTieCap;
                        const uint32_t gxy = (uint32_t)(wrapi(o[0] + x, L0) * L1 + wrapi(o[1] + y, L1));
                        for (int rb = 0; rb < total; rb += kWaveTieCap) {
                            int slot = below - rb;
                            uint32_t t2 = Tm;
                            while (t2) {
                                const int j = __ffs(t2) - 1;
                                t2 &= t2 - 1;
                                if ((unsigned)slot < (unsigned)kWaveTieCap)
                                    seg[slot] = make_uint2((uint32_t)row | ((uint32_t)(2 * j + zo) << 16) |
                                                               (((I >> j) & 1u) << 22),
                                                           gxy);
                                ++slot;
                            }
                            // LDS operations of one wavefront complete in order: keep
                            // the compiler from moving the reads above the writes
                            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                            __builtin_amdgcn_wave_barrier();
                            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                            const int nt = min(total - rb, kWaveTieCap);
                            auto draw = [&](const uint2 en) {
                                const int tz = (int)((en.x >> 16) & 63u);
                                const uint32_t site = en.y * (uint32_t)L2 + (uint32_t)wrapi(o[2] + tz, L2);
                                if (rng_bit(seed, site, sweep, Lt.instance_id, (uint32_t)r)) {
                                    atomicXor(Sc + (en.x & 0xFFFFu) * RS, 1u << (tz >> 1));
                                    nflip += (int)(en.x >> 22);
                                }
                            };
                            if (lane < nt) draw(seg[lane]);
                            if (lane + 64 < nt) draw(seg[lane + 64]);
                            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                            __builtin_amdgcn_wave_barrier();
                            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                        }
                    }
                } else {
                    if (ns != s) wc[2 * kPlS] = ns;
                }
            }
            if constexpr (CONV) {
                if (c == 1) {
                    // the sweep's last colour: report arrival and whether the interior flipped
                    const int any = __syncthreads_or(fsw != 0u);
                    fsw = 0;
                    if (tid == 0) {
                        // the returned value is used (a counter never reaches its top
                        // bit), so the add has completed before this tile's later
                        // stores, its next exchange words, are issued
                        const unsigned long long old =
                            atomicAdd((unsigned long long*)(sc + (p >> 1)), (1ull << 32) | (any ? 1ull : 0ull));
                        if (old >> 63) __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                } else {
                    __syncthreads();
                }
            } else {
                __syncthreads();
            }
        }
        // ---- exchange: publish the interior z-rows, then read the box back.
        // Every word travels with the epoch's tag in one 8-byte agent-scope
        // atomic, so a reader that sees the tag holds the word of this epoch
        // and no separate flag is needed.  Reuse of a buffer two epochs later
        // is safe: a tile publishes into it again only after reading words of
        // the next epoch from every neighbour (the boxes overlap both ways),
        // and a neighbour publishes those only after it has read this epoch's.
        uint64_t* gw = (e & 1) ? g1 : g0;
        const uint64_t tag = (uint64_t)(uint32_t)(e + 1) << 32;
        for (int row = tid; row < nrow_int; row += kMscThreads) {
            const int x = (int)fdiv((uint32_t)row, mX1);
            const int y = row - x * X[1];
            const int bx = x + hk[0], by = y + hk[1];
            const int brow = bx * B[1] + by;
            const int pr = (par0 + bx + by) & 1;
            const uint64_t v = spread32(pw(kPlS, pr, brow)) | (spread32(pw(kPlS, pr ^ 1, brow)) << 1);
            const uint32_t w = (uint32_t)(v >> hk[2]) & low_bits(X[2]);
            __hip_atomic_store(gw + (int64_t)tile * rows_per_tile + row, tag | w, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();  // the reads below overwrite plane rows published above
        // After the last epoch the words are still awaited and written too:
        // then every neighbour has finished reading its box from the spin
        // array before this tile writes its interior back, and the box holds
        // the final neighbours of every interior site for the energy.
#pragma unroll
        for (int m = 0; m < kExRows; ++m) {
            const int row = tid + m * kMscThreads;
            if (row >= rows || failed) continue;
            const int x = (int)fdiv((uint32_t)row, mB1);
            const int y = row - x * B[1];
            uint64_t* const src = gw + exoff[m];
            uint64_t* al = src + (int64_t)tzm * rows_per_tile;
            uint64_t* ah = src + (int64_t)tzp * rows_per_tile;
            uint64_t* am = src + (int64_t)tc[2] * rows_per_tile;
            uint64_t pl = __hip_atomic_load(al, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            uint64_t ph = __hip_atomic_load(ah, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            uint64_t pm = __hip_atomic_load(am, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // bounded wait for the three words of this epoch; a timeout here or
            // in any other tile raises the error flag and ends every workgroup
            uint32_t left = 1u << 20;
            while (((pl ^ tag) | (ph ^ tag) | (pm ^ tag)) >> 32) {
                if (--left == 0 ||
                    ((left & 63u) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)) {
                    __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    failed = true;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
                if ((pl ^ tag) >> 32) pl = __hip_atomic_load(al, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if ((ph ^ tag) >> 32) ph = __hip_atomic_load(ah, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if ((pm ^ tag) >> 32) pm = __hip_atomic_load(am, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            if (failed) continue;
            const uint32_t wl = (uint32_t)pl, wh = (uint32_t)ph, wm = (uint32_t)pm;
            const uint64_t v = (uint64_t)((wl >> (Xzm - hk[2])) & low_bits(hk[2])) | ((uint64_t)wm << hk[2]) |
                               ((uint64_t)(wh & low_bits(hk[2])) << (hk[2] + X[2]));
            const int pr = (par0 + x + y) & 1;
            pw(kPlS, pr, row) = even32(v);
            pw(kPlS, pr ^ 1, row) = even32(v >> 1);
        }
        failed = __syncthreads_or(failed);
        if (failed) break;
        if constexpr (CONV) {
            // after this exchange's reads: the counters of sweeps s_next .. s_next + 63
            if (wave == 0 && s_stop == 0x7FFFFFFF) {
                const int s0 = s_next;
                const int sw = s0 + lane;
                const bool inb = sw < T;
                const uint64_t v = inb ? __hip_atomic_load(sc + sw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0ull;
                const bool complete = inb && (uint32_t)(v >> 32) >= (uint32_t)ntiles;
                const uint64_t cm = __ballot(complete);
                const uint64_t zm = __ballot(complete && (uint32_t)v == 0u);
                const int pre = cm == ~0ull ? 64 : __builtin_ctzll(~cm);  // completed prefix
                const uint64_t zp = pre == 64 ? zm : (zm & ((1ull << pre) - 1ull));
                if (lane == 0) {
                    if (zp) {
                        const int sstar = s0 + __builtin_ctzll(zp);
                        s_stop = (2 * sstar + 1) / k + drift + 2;
                    } else {
                        s_next = s0 + pre;
                    }
                }
            }
            __syncthreads();
            if (e + 1 >= s_stop) break;
        }
    }
    // write the interior back in internal order (one wavefront per row, lane = z)
    if (!failed) {
        for (int row = wave; row < nrow_int; row += kMscWaves) {
            const int x = (int)fdiv((uint32_t)row, mX1);
            const int y = row - x * X[1];
            const int bx = x + hk[0], by = y + hk[1];
            const int brow = bx * B[1] + by;
            const int z = lane;
            if (z < X[2]) {
                const int zb = hk[2] + z;
                const int c = (par0 + bx + by + zb) & 1;
                const uint32_t bit = (pw(kPlS, c, brow) >> (zb >> 1)) & 1u;
                const int g = gsite(bx, by, zb);
                cs[c * half + (g >> 1)] = (int8_t)(bit ? -1 : 1);
            }
        }
    }
    // exact energy of the interior from the final box (thread per interior row)
    long long eT = 0;
    if (!failed) {
        const uint32_t im0 = bit_range((hk[2] + 1) >> 1, (hk[2] + X[2] - 1) >> 1);
        const uint32_t im1 = bit_range(hk[2] >> 1, (hk[2] + X[2] - 2) >> 1);
        for (int row = tid; row < nrow_int; row += kMscThreads) {
            const int x = (int)fdiv((uint32_t)row, mX1);
            const int y = row - x * X[1];
            const int bx = x + hk[0], by = y + hk[1];
            const int brow = bx * B[1] + by;
            int e = 0;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int zo = (c - par0 - bx - by) & 1;
                const uint32_t* const wc = lds32 + brow * RS + c;
                const uint32_t* const wo = lds32 + brow * RS + (c ^ 1);
                const uint32_t s = wc[2 * kPlS], on = wo[2 * kPlS];
                const uint32_t I = zo ? im1 : im0;
                // unsatisfied +y and +z bonds (and +x in 3-D)
                int u = __popc((s ^ wo[RS + 2 * kPlS] ^ wc[2 * kPlJY]) & I) +
                        __popc((s ^ (zo ? (on >> 1) : on) ^ wc[2 * kPlJZ]) & I);
                if constexpr (D == 3) u += __popc((s ^ wo[B[1] * RS + 2 * kPlS] ^ wc[2 * kPlJX]) & I);
                const uint32_t hp = wc[2 * kPlHP], hn = wc[2 * kPlHN], ha = wc[2 * kPlHA];
                const uint32_t gpos = (hp & ~s) | (hn & s);
                const uint32_t gneg = (hn & ~s) | (hp & s);
                const int sg = __popc(gpos & I) + __popc(gpos & ha & I) - __popc(gneg & I) - __popc(gneg & ha & I);
                e += 2 * u - D * __popc(I) - sg;
            }
            eT += e;
        }
    }
    long long nf = nflip;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        eT += __shfl_xor(eT, off, 64);
        nf += __shfl_xor(nf, off, 64);
    }
    __shared__ long long pd[kMscWaves], pf[kMscWaves];
    if (lane == 0) {
        pd[wave] = eT;
        pf[wave] = nf;
    }
    __syncthreads();
    if (tid == 0) {
        long long a = 0, b2 = 0;
        for (int w = 0; w < kMscWaves; ++w) {
            a += pd[w];
            b2 += pf[w];
        }
        int64_t* ap = acc + 2 * ((int64_t)r * nslots + tile);
        ap[0] = a;  // the tile's energy (absolute)
        ap[1] += b2;
    }
}

// ---------------------------------------------------------------------------

static void msc_box(const TileGeom& tg, const int L[3], int D, int B[3])
{
    for (int a = 0; a < 3; ++a) {
        const int mx = (L[a] + tg.P[a] - 1) / tg.P[a];
        B[a] = mx + ((D == 2 && a == 0) ? 0 : 2 * tg.k);
    }
}

size_t lattice_msc_lds(const TileGeom& tg, const int L[3], int D)
{
    int B[3];
    msc_box(tg, L, D, B);
    const size_t words = ((size_t)(2 * msc_planes(D) + 1) * B[0] * B[1] + 1) & ~(size_t)1;
    return words * 4 + (size_t)kMscWaves * kWaveTieCap * 8;
}

bool lattice_msc_geometry_ok(const TileGeom& tg, const int L[3], int D)
{
    int B[3];
    msc_box(tg, L, D, B);
    if (tg.k < 1 || tg.k > 62) return false;
    if (B[2] > 64) return false;                           // a box z-row is two 32-bit colour words
    if ((L[2] + tg.P[2] - 1) / tg.P[2] > 32) return false;  // an interior z-row is one exchange word
    if ((int64_t)B[0] * B[1] > 65535) return false;        // tie queue entries hold the row in 16 bits
    if ((int64_t)B[0] * B[1] > kExRows * kMscThreads) return false;  // exchange offsets held in registers
    for (int a = (D == 2 ? 1 : 0); a < 3; ++a)
        if (L[a] / tg.P[a] < tg.k) return false;           // the halo stays within the 26 neighbour tiles
    return true;
}

template <int D, bool TIE, bool CONV>
static const void* msc_kernel() { return (const void*)k_lattice_msc<D, TIE, CONV>; }

static const void* pick_msc_kernel(int D, bool tie, bool conv)
{
    if (conv) return D == 3 ? msc_kernel<3, false, true>() : msc_kernel<2, false, true>();
    return D == 3 ? (tie ? msc_kernel<3, true, false>() : msc_kernel<3, false, false>())
                  : (tie ? msc_kernel<2, true, false>() : msc_kernel<2, false, false>());
}

// The replica's sweep count under the stopping rule, from the counters of
// its tiles (after the launch): lastflip = done + the first sweep that every
// tile reached without a flip, or done + T when there is none.  A replica
// whose lastflip is below done converged in an earlier chunk and is left.
__global__ void k_msc_settle(RepState* __restrict__ rs, int R, const uint64_t* __restrict__ scnt, int T, int done,
                             int ntiles)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    RepState* st = rs + r;
    if (st->converged || st->lastflip < done) return;
    const uint64_t* sc = scnt + (int64_t)r * T;
    int first = T;
    for (int s = 0; s < T; ++s) {
        const uint64_t v = sc[s];
        if ((uint32_t)(v >> 32) < (uint32_t)ntiles) break;
        if ((uint32_t)v == 0u) {
            first = s;
            break;
        }
    }
    st->lastflip = done + first;
}

hipError_t launch_lattice_msc(const LatticeDev& Lt, const TileGeom& tg, int8_t* canon, int64_t stride, uint64_t* G0,
                              uint64_t* G1, uint32_t* err, RepState* rs, int R, int64_t* acc,
                              int nslots, int T, uint64_t seed, int rule, hipStream_t st, uint64_t* scnt, int done)
{
    if (!lattice_msc_geometry_ok(tg, Lt.L, Lt.D)) return hipErrorInvalidValue;
    const bool conv = scnt != nullptr;
    if (conv && rule == 1) return hipErrorInvalidValue;
    const void* kern = pick_msc_kernel(Lt.D, rule == 1, conv);
    const size_t lds = lattice_msc_lds(tg, Lt.L, Lt.D);
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const int ntiles = tg.P[0] * tg.P[1] * tg.P[2];
    // the largest distance between two tiles on the torus of tiles (Chebyshev)
    int drift = 0;
    for (int a = 0; a < 3; ++a) drift = std::max(drift, tg.P[a] / 2);
    LatticeDev a0 = Lt;
    TileGeom a1 = tg;
    void* args[] = {&a0, &a1, &canon, &stride, &G0, &G1, &err, &rs, &acc, &nslots, &T, &seed, &scnt, &drift};
    e = hipLaunchCooperativeKernel(kern, dim3(ntiles * R), dim3(kMscThreads), args, (unsigned)lds, st);
    if (e != hipSuccess || !conv) return e;
    hipLaunchKernelGGL(k_msc_settle, dim3((R + 63) / 64), dim3(64), 0, st, rs, R, (const uint64_t*)scnt, T, done,
                       ntiles);
    return hipGetLastError();
}

int lattice_msc_max_blocks(const TileGeom& tg, const int L[3], int D)
{
    const void* kern = pick_msc_kernel(D, true, false);
    const size_t lds = lattice_msc_lds(tg, L, D);
    int per_cu = 0, dev = 0, cus = 0;
    if (hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kMscThreads, lds) != hipSuccess ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return per_cu * cus;
}

}  // namespace sg
