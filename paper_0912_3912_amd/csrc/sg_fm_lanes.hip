// sg_fm_lanes.hip -- the paper's pass-based local search with hill-climbing
// (Sec. IV, Fig. 3), one replica per lane.
//
// The moves of one pass form a serial chain, so a replica cannot be spread
// over a wavefront without paying a wave-wide selection and a wave-wide
// update for every move.  Here every lane runs its own replica instead: the
// lanes of a workgroup take restarts of one instance, and every lane makes
// one move per step of the loop.  Every pass has exactly n moves (each spin
// is moved once and then locked), so the lanes of a wavefront reach their
// pass boundaries together; a lane whose replica has finished takes the
// next restart of the workgroup's item there (one atomic counter per item,
// shared by the workgroup's wavefronts).
//
// Per lane, in its wavefront's LDS (word k of lane l at k*64 + l, so that
// the lanes of one access always hit 64 different banks):
//   gains   one byte per spin, external order: 0 for a locked spin, else
//           v + 128 where v = -s_i f_i is half the gain -dE_i of moving i
//           (every |f_i| <= 127: the host admits only instances whose
//           per-spin sum of |coefficients| is at most 127);
//   spins   one bit per spin (1: s = -1);
//   bests   per group of 32 spins, the largest key (v + 128) << 16 |
//           (65535 - i) of its spins: larger gain first, then lower external
//           index; exact for every group not marked for a rescan.
// A move takes the largest of the group keys, locks and flips the spin,
// updates the half-gains of its unlocked partners (a flip of s_i changes f_j
// by -2 J_ij s_i and f_a by -2 K s_i s_b) and rescans the groups it touched:
// a rescan packs the group's 32 gain bytes into 16-bit keys (gain byte,
// 255 - position) two at a time and takes their maximum with packed 16-bit
// maxima.  The instance's term rows (fixed width per instance, external
// order) are read from device memory; they are shared by all lanes and stay
// in the caches.
//
// The move order that undoes the moves after the best prefix is kept as a
// tag per spin in the replica's own spin row in device memory (free while
// the pass runs): tag = step >> sh (sh = 0, 1, 2 for n <= 256, 512, 1024), so
// a spin is kept iff its tag is below the block of the last kept step, or it
// is one of the moves of that block up to the last kept step, which a shift
// register of the last four moves records whenever the energy reaches a new
// low.  Counters and the stopping rule are those of the wavefront-per-replica
// kernel: sweeps += passes, flips += moves kept, attempts = passes x n; under
// until_converged a replica stops after the first pass that does not lower
// the energy of its best state (that pass counts).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sg_launch.h"
#include "sg_layout.h"

namespace sg {

constexpr int kFmlMaxN = 1024;

typedef unsigned short fml_u16x2 __attribute__((ext_vector_type(2)));
// device-memory views (the pointers come from the instance table, so the
// compiler would otherwise address them as generic memory)
typedef uint32_t fml_v2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) const fml_v2 fml_g2;
typedef __attribute__((address_space(1))) const uint32_t fml_g32;
typedef __attribute__((address_space(1))) int8_t fml_gi8;
typedef __attribute__((address_space(1))) uint32_t fml_gu32;
// read-only views for loads at wavefront-uniform addresses (scalar loads)
typedef __attribute__((address_space(4))) const fml_v2 fml_k2;
typedef __attribute__((address_space(4))) const uint32_t fml_k32;

// LDS of one wavefront: gain words for whole groups (8 per group), spin
// words (1 per group) and group keys (a multiple of 8), 64 lanes each.
size_t fml_wave_lds_bytes(int nmax)
{
    const size_t g = ((size_t)nmax + 31) / 32, gp = (g + 7) / 8 * 8;
    return 256 * (8 * g + g + gp);
}

// bytes 255 - 4d - u (u = 0..3): the position part of a group's 16-bit keys
__device__ __forceinline__ uint32_t fml_pos_bytes(int d)
{
    const uint32_t b = 255u - 4u * (uint32_t)d;
    return b | (b - 1u) << 8 | (b - 2u) << 16 | (b - 3u) << 24;
}

// Spin j's byte offset in the lane-interleaved gain words (the lane's own
// four bytes of word j/4 sit at (j/4)*256 + lane*4): fb(j) = (j >> 2) * 256 +
// (j & 3).  fb grows with j, so 65535 - fb(j) orders equal gains by lower
// index, and j >> 5 (its group and spin word) is fb >> 11.
__device__ __forceinline__ int fml_spin_of(uint32_t fb) { return (int)(((fb >> 8) << 2) | (fb & 3u)); }

// The largest key of group g of this lane (gain words 8g .. 8g + 7; the
// bytes of spins at or beyond n are zero, as locked), as gain byte << 16 |
// (65535 - fb).
__device__ __forceinline__ uint32_t fml_group_key(const uint32_t* gw, int g, int lane)
{
    const uint32_t* p = gw + g * 8 * 64 + lane;
    uint32_t x[8];
#pragma unroll
    for (int d = 0; d < 8; ++d) x[d] = p[d * 64];
    fml_u16x2 m = {0, 0};
#pragma unroll
    for (int d = 0; d < 8; ++d) {
        const uint32_t c = fml_pos_bytes(d);
        const uint32_t lo = __builtin_amdgcn_perm(x[d], c, 0x05010400u);  // (byte 0, pos 0), (byte 1, pos 1)
        const uint32_t hi = __builtin_amdgcn_perm(x[d], c, 0x07030602u);  // (byte 2, pos 2), (byte 3, pos 3)
        m = __builtin_elementwise_max(m, __builtin_bit_cast(fml_u16x2, lo));
        m = __builtin_elementwise_max(m, __builtin_bit_cast(fml_u16x2, hi));
    }
    const uint32_t k16 = m.x > m.y ? m.x : m.y;
    const uint32_t p32 = 255u - (k16 & 0xFFu);  // position in the group
    const uint32_t fb = (uint32_t)g * 2048u + (p32 >> 2) * 256u + (p32 & 3u);
    return (k16 >> 8) << 16 | (0xFFFFu - fb);
}

// Row layout (InstTab::fml): per spin a word h & 255 | couplings << 8 |
// hyper-couplings << 16 (padded to an even count), then DC coupling words
// per spin, each fb(j) << 16 | (j & 31) << 11 | J & 255, then TT pairs of
// words per spin, one hyper-coupling each: (fb(a) << 16 | fb(b), (a & 31) <<
// 24 | (b & 31) << 16 | K & 255).  Unused entries name the spin itself with
// coefficient 0.  DC (4, 6, 8 or 16) and TT (0, 2, 4 or 6) are the row widths
// of every instance of a launch: fixed at compile time, so that a row's loads
// are issued together.
template <int DC, int TT>
__global__ __launch_bounds__(256) void k_fm_lanes(const InstTab* __restrict__ tab, BlockItem* __restrict__ items,
                                                  int wave_words, RepState* __restrict__ rs,
                                                  CallStats* __restrict__ cs, uint32_t* __restrict__ err,
                                                  int max_passes, int until_conv)
{
    extern __shared__ uint32_t fml_lds[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const BlockItem it = items[blockIdx.x];
    uint32_t* counter = reinterpret_cast<uint32_t*>(&items[blockIdx.x].pad);
    const InstTab& Q = tab[it.inst];
    const int n = Q.I.n;
    const int G = (n + 31) >> 5, Gp = (G + 7) & ~7;
    const int sh = n <= 256 ? 0 : (n <= 512 ? 1 : 2);
    uint32_t* gw = fml_lds + (size_t)wave * wave_words;  // gain bytes, word w of lane l at w*64 + l
    uint32_t* sw = gw + G * 8 * 64;                       // spin bits
    uint32_t* bw = sw + G * 64;                           // group keys (Gp, zero beyond G)
    uint8_t* gl8 = reinterpret_cast<uint8_t*>(gw + lane);  // this lane's gain byte of spin j at gl8[fb(j)]
    uint32_t* sl = sw + lane;                              // this lane's spin word k at sl[k * 64]
    uint32_t* bl = bw + lane;                              // this lane's group key g at bl[g * 64]
    constexpr int TTa = TT > 0 ? TT : 1;
    fml_g32* hg = (fml_g32*)Q.fml;
    fml_g2* cw2 = (fml_g2*)(Q.fml + ((n + 1) & ~1));
    fml_g2* tw2 = cw2 + (size_t)n * (DC / 2);
    fml_k32* ext = (fml_k32*)Q.I.ext;
    fml_k32* hk = (fml_k32*)Q.fml;
    fml_k2* ck2 = (fml_k2*)(Q.fml + ((n + 1) & ~1));
    fml_k2* tk2 = ck2 + (size_t)n * (DC / 2);

    auto sgn = [&](int j) { return ((sl[(j >> 5) * 64] >> (j & 31)) & 1u) ? -1 : 1; };

    int r = -1;              // restart of this lane's replica, -1: none
    bool drained = false;    // the item has no restarts left (wave-uniform)
    bool bad = false;
    RepState* st = nullptr;
    fml_gi8* gs = nullptr;
    long long Estar = 0, kept = 0;
    int pc = 0;
    long long att_all = 0, kept_all = 0;
    int passes_max = 0, unconv = 0;

    for (;;) {
        // hand the item's next restarts to the idle lanes
        while (!drained) {
            const uint64_t idle = __ballot(r < 0 && !bad);
            if (idle == 0) break;
            const int rank =
                (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(idle >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)idle, 0u));
            int first = 0;
            if (lane == __builtin_ctzll(idle)) first = (int)atomicAdd(counter, (uint32_t)__popcll(idle));
            first = __builtin_amdgcn_readlane(first, __builtin_ctzll(idle));
            if (first + __popcll(idle) >= it.nr) drained = true;
            bool fresh = false;
            if (r < 0 && !bad) {
                const int c = first + rank;
                if (c < it.nr) {
                    RepState* s2 = rs + Q.rep_base + it.r0 + c;
                    if (!s2->converged) {
                        r = it.r0 + c;
                        st = s2;
                        fresh = true;
                    }
                }
            }
            if (__ballot(fresh)) {
                if (fresh) {
                    gs = (fml_gi8*)(Q.spins + Q.spin_stride * r);
                    Estar = st->E;
                    pc = 0;
                    kept = 0;
                    for (int g = 0; g < G; ++g) sl[g * 64] = 0u;
                }
                for (int i0 = 0; i0 < n; i0 += 4) {
                    const uint32_t w4 = fresh ? *(const fml_gu32*)(gs + i0) : 0u;
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int i = i0 + u;
                        if (i < n) {
                            const int e = (int)ext[i];
                            if (fresh && (int8_t)(w4 >> (8 * u)) < 0) atomicOr(&sl[(e >> 5) * 64], 1u << (e & 31));
                        }
                    }
                }
            }
        }
        if (__ballot(r >= 0) == 0) break;
        const bool act = r >= 0;

        // half-gains from the definition, and the group keys; the lane's spin
        // words sit in registers (indexed by the wavefront-uniform partner)
        if (act) {
            uint32_t sreg[32];
#pragma unroll
            for (int g = 0; g < 32; ++g) sreg[g] = g < G ? sl[g * 64] : 0u;
            auto sr = [&](uint32_t wi, uint32_t bi) { return ((sreg[wi] >> bi) & 1u) ? -1 : 1; };
            for (int g = G; g < Gp; ++g) bl[g * 64] = 0u;
            for (int g = 0; g < G; ++g) {
                uint32_t best = 0;
                for (int d = 0; d < 8; ++d) {
                    uint32_t word = 0;
                    const int e0 = g * 32 + d * 4;
                    // the four spins' rows, every load issued before any is used
                    int hq[4];
                    fml_v2 cr[4][DC / 2], tr[4][TTa];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int e = e0 + u < n ? e0 + u : n - 1;
                        hq[u] = (int)hk[e];
#pragma unroll
                        for (int c = 0; c < DC / 2; ++c) cr[u][c] = ck2[(size_t)e * (DC / 2) + c];
#pragma unroll
                        for (int c = 0; c < TT; ++c) tr[u][c] = tk2[(size_t)e * TT + c];
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int e = e0 + u;
                        if (e < n) {
                            // the row's counts are wavefront-uniform: unused entries are skipped
                            const int nc = (hq[u] >> 8) & 0xFF, nt = hq[u] >> 16;
                            int f = (int)(int8_t)(hq[u] & 0xFF);
#pragma unroll
                            for (int c = 0; c < DC / 2; ++c) {
                                const uint32_t wq[2] = {cr[u][c].x, cr[u][c].y};
#pragma unroll
                                for (int k = 0; k < 2; ++k)
                                    if (2 * c + k < nc)
                                        f += (int)(int8_t)(wq[k] & 0xFFu) * sr(wq[k] >> 27, (wq[k] >> 11) & 31u);
                            }
#pragma unroll
                            for (int c = 0; c < TT; ++c) {
                                const uint32_t w0 = tr[u][c].x, w1 = tr[u][c].y;
                                if (c < nt)
                                    f += (int)(int8_t)(w1 & 0xFFu) * sr(w0 >> 27, (w1 >> 24) & 31u) *
                                         sr((w0 & 0xFFFFu) >> 11, (w1 >> 16) & 31u);
                            }
                            const uint32_t vb = (uint32_t)(128 - sr((uint32_t)e >> 5, (uint32_t)e & 31u) * f);
                            word |= vb << (8 * u);
                            const uint32_t key = vb << 16 | (0xFFFFu - (uint32_t)(g * 2048 + d * 256 + u));
                            best = key > best ? key : best;
                        }
                    }
                    gw[(g * 8 + d) * 64 + lane] = word;
                }
                bl[g * 64] = best;
            }
        }

        // the n moves of the pass; top is the largest group key
        long long E = Estar, Elow = Estar;
        int blen = 0;
        uint64_t ring = 0, saved = 0;
        uint32_t top = 0;
        for (int g0 = 0; g0 < Gp; g0 += 8) {
            uint32_t b[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) b[u] = bl[(g0 + u) * 64];
#pragma unroll
            for (int u = 0; u < 8; ++u) top = b[u] > top ? b[u] : top;
        }
        for (int step = 0; step < n; ++step) {
            if (!act || bad) continue;
            const int vb = (int)(top >> 16);
            if (vb == 0) {  // no unlocked spin left before n moves: internal error, stop this replica
                bad = true;
                continue;
            }
            const uint32_t fe = 0xFFFFu - (top & 0xFFFFu);
            const int e = fml_spin_of(fe);
            // the spin's rows: loads issued before anything waits on them
            fml_g2* crow = cw2 + (size_t)e * (DC / 2);
            fml_g2* trow = tw2 + (size_t)e * TT;
            fml_v2 cq[DC / 2], tq[TTa];
            const uint32_t hw = TT > 0 ? hg[e] : 0u;
#pragma unroll
            for (int c = 0; c < DC / 2; ++c) cq[c] = crow[c];
#pragma unroll
            for (int c = 0; c < TT; ++c) tq[c] = trow[c];
            gs[e] = (int8_t)(step >> sh);  // the move's tag
            gl8[fe] = 0;                   // locked
            uint32_t* sp = &sl[(fe >> 11) * 64];
            const uint32_t sword = *sp;
            ring = ring << 16 | (uint32_t)e;
            E -= 2 * (vb - 128);
            if (E < Elow) {
                Elow = E;
                blen = step + 1;
                saved = ring;
            }
            // every read of the partners' state issued together (an unused
            // entry names spin e itself, now locked, with coefficient 0: it
            // changes nothing), then every change computed, then written
            uint32_t gbv[DC], spv[DC], kv[DC];
            uint32_t sa[TTa], sb[TTa], la[TTa], lb[TTa];
#pragma unroll
            for (int c = 0; c < DC / 2; ++c) {
                const uint32_t wq[2] = {cq[c].x, cq[c].y};
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    const uint32_t fb = wq[k] >> 16;
                    gbv[2 * c + k] = gl8[fb];
                    spv[2 * c + k] = sl[(fb >> 11) * 64];
                    kv[2 * c + k] = bl[(fb >> 11) * 64];
                }
            }
            // hyper-coupling slots that some lane uses (the rest are skipped)
            int tmax = 0;
#pragma unroll
            for (int c = 0; c < TT; ++c)
                if (__ballot((int)(hw >> 16) > c)) tmax = c + 1;
#pragma unroll
            for (int c = 0; c < TT; ++c) {
                if (c < tmax) {
                    const uint32_t fa = tq[c].x >> 16, fbb = tq[c].x & 0xFFFFu;
                    sa[c] = sl[(fa >> 11) * 64];
                    sb[c] = sl[(fbb >> 11) * 64];
                    la[c] = gl8[fa];
                    lb[c] = gl8[fbb];
                }
            }
            const int s_old = ((sword >> (e & 31)) & 1u) ? -1 : 1;
            const int m2 = 2 * s_old;  // a partner's half-gain changes by J * m2 * s_j
            *sp = sword ^ (1u << (e & 31));
            uint32_t dirty = 1u << (fe >> 11);
            // couplings (distinct partners): a raised key raises its group's; a
            // lowered one that was the group's largest before this move asks
            // for a rescan
#pragma unroll
            for (int c = 0; c < DC / 2; ++c) {
                const uint32_t wq[2] = {cq[c].x, cq[c].y};
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    const uint32_t w = wq[k], fb = w >> 16, b = gbv[2 * c + k];
                    const int dj = (int)(int8_t)(w & 0xFFu) * m2;
                    const int dv = ((spv[2 * c + k] >> ((w >> 11) & 31u)) & 1u) ? -dj : dj;
                    const uint32_t nb = b ? (uint32_t)((int)b + dv) : 0u;  // a locked partner keeps 0
                    const uint32_t lo = 0xFFFFu - fb;
                    dirty |= (nb < b && kv[2 * c + k] == (b << 16 | lo)) ? 1u << (fb >> 11) : 0u;
                    gl8[fb] = (uint8_t)nb;
                    atomicMax(&bl[(fb >> 11) * 64], nb << 16 | lo);
                }
            }
            // hyper-couplings: a spin may sit in several, so the half-gains
            // change by atomic adds on their words (each byte's value before
            // and after all of a move's changes lies in 1..255, so the adds of
            // the whole word carry nothing into a neighbouring byte at the
            // end); their groups are rescanned
#pragma unroll
            for (int c = 0; c < TT; ++c) {
                if (c < tmax) {
                    const uint32_t w0 = tq[c].x, w1 = tq[c].y;
                    const uint32_t fa = w0 >> 16, fbb = w0 & 0xFFFFu;
                    const bool na = (sa[c] >> ((w1 >> 24) & 31u)) & 1u;
                    const bool nbn = (sb[c] >> ((w1 >> 16) & 31u)) & 1u;
                    const int dv = (int)(int8_t)(w1 & 0xFFu) * m2 * (na != nbn ? -1 : 1);
                    atomicAdd(reinterpret_cast<uint32_t*>(gl8 + (fa & ~3u)),
                              la[c] ? (uint32_t)dv << (8 * (fa & 3u)) : 0u);
                    atomicAdd(reinterpret_cast<uint32_t*>(gl8 + (fbb & ~3u)),
                              lb[c] ? (uint32_t)dv << (8 * (fbb & 3u)) : 0u);
                    dirty |= 1u << (fa >> 11) | 1u << (fbb >> 11);
                }
            }
            // the next move's key: the touched groups' keys are set aside (zero),
            // every key is read in the same round trip as the rescan's gain
            // words, and the rescanned keys join the maximum
            for (uint32_t z = dirty; z; z &= z - 1u) bl[__builtin_ctz(z) * 64] = 0u;
            top = 0;
            for (int g0 = 0; g0 < Gp; g0 += 8) {
                uint32_t b[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) b[u] = bl[(g0 + u) * 64];
#pragma unroll
                for (int u = 0; u < 8; ++u) top = b[u] > top ? b[u] : top;
            }
            // rescan the touched groups: one when no lane has touched more,
            // else two at a time
            if (!__ballot(__popc(dirty) > 1)) {
                const int g1 = __builtin_ctz(dirty);
                const uint32_t k1 = fml_group_key(gw, g1, lane);
                bl[g1 * 64] = k1;
                top = k1 > top ? k1 : top;
                dirty = 0;
            }
            while (dirty) {
                const int g1 = __builtin_ctz(dirty);
                dirty &= dirty - 1u;
                const int g2 = dirty ? __builtin_ctz(dirty) : g1;
                dirty &= dirty - 1u;
                const uint32_t k1 = fml_group_key(gw, g1, lane);
                const uint32_t k2 = fml_group_key(gw, g2, lane);
                bl[g1 * 64] = k1;
                bl[g2 * 64] = k2;
                top = k1 > top ? k1 : top;
                top = k2 > top ? k2 : top;
            }
        }

        // the pass ends: keep the best prefix, then finish or go on
        if (act && !bad) {
            // every spin moved once in the pass: flip back those after the prefix
            const int T = blen > 0 ? (blen - 1) >> sh : -1;
            for (int g = 0; g < G; ++g) {
                uint32_t t4[8];
#pragma unroll
                for (int d = 0; d < 8; ++d) {
                    const int e0 = g * 32 + d * 4;
                    t4[d] = e0 < n ? *(const fml_gu32*)(gs + e0) : 0u;
                }
                uint32_t keep = 0;
#pragma unroll
                for (int d = 0; d < 8; ++d)
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        if ((int)((t4[d] >> (8 * u)) & 0xFFu) < T) keep |= 1u << (d * 4 + u);
                const int rem = n - g * 32;
                const uint32_t valid = rem >= 32 ? 0xFFFFFFFFu : (1u << rem) - 1u;
                sl[g * 64] ^= ~keep & valid;
            }
            if (blen > 0) {
                // the moves of the last kept step's block up to that step (tag T) were flipped back above
                const int c = ((blen - 1) & ((1 << sh) - 1)) + 1;
                for (int q = 0; q < c; ++q) {
                    const int e = (int)((saved >> (16 * q)) & 0xFFFFu);
                    sl[(e >> 5) * 64] ^= 1u << (e & 31);
                }
            }
            ++pc;
            kept += blen;
            const bool improved = Elow < Estar;
            Estar = Elow;
            const bool conv = until_conv && !improved;
            if (conv || pc >= max_passes) {
                for (int i0 = 0; i0 < n; i0 += 4) {
                    uint32_t w4 = 0;
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int i = i0 + u;
                        if (i < n) w4 |= (sgn((int)ext[i]) < 0 ? 0xFFu : 0x01u) << (8 * u);
                    }
                    if (i0 + 3 < n) {
                        *(fml_gu32*)(gs + i0) = w4;
                    } else {
                        for (int u = 0; i0 + u < n; ++u) gs[i0 + u] = (int8_t)(w4 >> (8 * u));
                    }
                }
                st->E = Estar;
                st->sweeps += pc;
                st->flips += kept;
                if (conv) st->converged = 1;
                else if (until_conv) ++unconv;
                att_all += (long long)pc * n;
                kept_all += kept;
                passes_max = pc > passes_max ? pc : passes_max;
                r = -1;
            }
        }
        if (bad) r = -1;
    }
    if (bad) atomicOr(err, 1u);
    // call totals: one atomic per wavefront
    for (int o = 32; o > 0; o >>= 1) {
        att_all += __shfl_xor(att_all, o);
        kept_all += __shfl_xor(kept_all, o);
        unconv += __shfl_xor(unconv, o);
        const int pm = __shfl_xor(passes_max, o);
        passes_max = pm > passes_max ? pm : passes_max;
    }
    if (lane == 0 && (att_all || unconv)) {
        atomicAdd(&cs->attempts, (unsigned long long)att_all);
        atomicAdd(&cs->flips, (unsigned long long)kept_all);
        atomicMax(&cs->sweeps_max, (unsigned long long)passes_max);
        atomicAdd(&cs->unconverged, (unsigned long long)unconv);
    }
}

// Wavefronts per workgroup (they share the item's restarts and the caches
// hold the instance's rows once for all of them): want (0: one) bounded by
// four and by the LDS; 0 when one wavefront's LDS exceeds the compute unit's.
int fml_waves_per_block(int nmax, int want)
{
    const size_t w = fml_wave_lds_bytes(nmax);
    int k = (int)((size_t)(160 * 1024) / w);
    if (k < 1) return 0;
    if (want <= 0) want = 1;
    k = k < want ? k : want;
    return k > 4 ? 4 : k;
}

template <int DC, int TT>
static const void* fml_kernel()
{
    return (const void*)k_fm_lanes<DC, TT>;
}

// the instantiation for row widths (dc, tt): dc in {4, 6, 8, 16}, tt in {0, 2, 4, 6}
static const void* fml_pick(int dc, int tt)
{
    switch (dc * 10 + tt) {
    case 40: return fml_kernel<4, 0>();
    case 42: return fml_kernel<4, 2>();
    case 44: return fml_kernel<4, 4>();
    case 46: return fml_kernel<4, 6>();
    case 60: return fml_kernel<6, 0>();
    case 62: return fml_kernel<6, 2>();
    case 64: return fml_kernel<6, 4>();
    case 66: return fml_kernel<6, 6>();
    case 80: return fml_kernel<8, 0>();
    case 82: return fml_kernel<8, 2>();
    case 84: return fml_kernel<8, 4>();
    case 86: return fml_kernel<8, 6>();
    case 160: return fml_kernel<16, 0>();
    case 162: return fml_kernel<16, 2>();
    case 164: return fml_kernel<16, 4>();
    case 166: return fml_kernel<16, 6>();
    default: return nullptr;
    }
}

int fml_resident_blocks(int nmax, int W, int dc, int tt)
{
    if (W <= 0) return 0;
    const void* kern = fml_pick(dc, tt);
    if (!kern) return 0;
    const size_t lds = fml_wave_lds_bytes(nmax) * (size_t)W;
    int per_cu = 0, dev = 0, cus = 0;
    if (hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, W * 64, lds) != hipSuccess ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return per_cu * cus;
}

hipError_t launch_fm_lanes(const InstTab* tab, BlockItem* items, int nitems, int nmax, int W, int dc, int tt,
                           RepState* rs, CallStats* cs, uint32_t* err, int max_passes, int until_conv, hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    const void* kern = fml_pick(dc, tt);
    if (!kern || nmax < 1 || nmax > kFmlMaxN || W < 1 || W > 4 || fml_wave_lds_bytes(nmax) * (size_t)W > 160 * 1024)
        return hipErrorInvalidValue;
    const size_t wave_bytes = fml_wave_lds_bytes(nmax);
    const size_t lds = wave_bytes * (size_t)W;
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    int wave_words = (int)(wave_bytes / 4);
    void* args[] = {(void*)&tab, (void*)&items, (void*)&wave_words, (void*)&rs, (void*)&cs, (void*)&err,
                    (void*)&max_passes, (void*)&until_conv};
    return hipLaunchKernel(kern, dim3(nitems), dim3(W * 64), args, lds, st);
}

}  // namespace sg
