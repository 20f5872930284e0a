// sg_lattice.hip -- colour-ordered sweeps on periodic 2-D/3-D lattices with
// implicit neighbours, LDS-resident.
//
// Sites are addressed (x, y, z) with z fastest (a 2-D lattice is stored as
// 1 x Lx x Ly and has no x bonds); all extents are even so the colouring is
// the checkerboard colour(g) = (x + y + z + c0) mod 2, identical to the
// colour-major relabel of the general path (internal index of site g =
// colour(g) * n/2 + g/2).  Each site carries one 64-bit record: the
// couplings to its +x, -x, +y, -y, +z, -z neighbours and its field, as int8.
//
// k_lattice_tiles: one workgroup per tile of the lattice (one launch for the
// whole run, all workgroups co-resident).  A workgroup keeps its tile plus a
// halo of width k in LDS and advances k colour phases between exchanges;
// after phase q of an epoch only sites at least q+1 layers inside the box are
// still exact (each update needs its six neighbours from the previous
// phase), so after k phases exactly the tile interior is exact.  It then
// publishes its interior as one 32-bit word per z-row (bit per spin), each
// stored with the epoch's tag in one 8-byte agent-scope atomic, and reads its
// new halo: at most three word loads per box row, all issued at once and each
// polled until its tag shows the epoch (no separate flag).  The exchange
// buffer alternates between two copies by epoch parity; a tile writes a copy
// again only after reading words of the next epoch from every neighbour, and
// a neighbour publishes those only after it has read this copy.  Each thread's sites are sorted deepest first,
// so phase q walks only the sites deeper than q.  Every wait is bounded: on
// time-out the kernel records an error and every workgroup exits.
//
// k_lattice_wg: the whole lattice of one replica in one workgroup (small
// lattices, many replicas); supports the per-replica stopping rule exactly.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

#include "sg_device.h"
#include "sg_launch.h"
#include "sg_layout.h"

namespace sg {

__device__ __forceinline__ int jb(uint64_t rec, int k) { return (int)(int8_t)(rec >> (8 * k)); }

constexpr int kLatThreads = 1024;
constexpr int kLatWaves = kLatThreads / 64;

// Per-thread site list entry: box index (bits 0..19), halo depth (bits
// 20..27: distance to the nearest box face over the axes that have a halo),
// valid flag (bit 28).
constexpr int kSiteValid = 1 << 28;
constexpr int kMaxDepth = 64;
__device__ __forceinline__ int site_b(int pk) { return pk & 0xFFFFF; }
__device__ __forceinline__ int site_depth(int pk) { return (pk >> 20) & 0xFF; }

template <int D, bool TIE, int NS>
__global__ __launch_bounds__(kLatThreads) void k_lattice_tiles(LatticeDev Lt, TileGeom tg, int8_t* __restrict__ canon,
                                                               int64_t stride, uint64_t* __restrict__ G0,
                                                               uint64_t* __restrict__ G1,
                                                               uint32_t* __restrict__ err, RepState* __restrict__ rs,
                                                               int64_t* __restrict__ acc, int nslots, int T,
                                                               uint64_t seed)
{
    extern __shared__ uint64_t lds64[];
    const int ntiles = tg.P[0] * tg.P[1] * tg.P[2];
    const int tile = blockIdx.x % ntiles;
    const int r = blockIdx.x / ntiles;
    // a replica frozen by an earlier call is not swept; all its tiles leave
    // together, and no other replica waits on them (exchanges are per replica)
    if (rs[r].converged) return;
    const int tid = threadIdx.x;
    const int L0 = Lt.L[0], L1 = Lt.L[1], L2 = Lt.L[2];
    const int n = Lt.n, half = n / 2;
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
    const int par0 = (((o[0] % 2) + (o[1] % 2) + (o[2] % 2) + Lt.c0) % 2 + 2) % 2;
    const int V = B[0] * B[1] * B[2];
    const int nint_all = X[0] * X[1] * X[2];
    const uint32_t mX1 = fdiv_magic((uint32_t)X[1]), mX2 = fdiv_magic((uint32_t)X[2]);
    const int nrow_int = X[0] * X[1], nrow_box = B[0] * B[1];
    // tile extents along an axis: start of tile t is floor(t L / P)
    auto tstart = [&](int a, int t) -> int { return (int)((int64_t)t * Lt.L[a] / tg.P[a]); };
    // z-neighbour tiles' extents (periodic)
    const int tzm = (tc[2] + tg.P[2] - 1) % tg.P[2], tzp = (tc[2] + 1) % tg.P[2];
    const int Xzm = tstart(2, tzm + 1) - tstart(2, tzm);
    uint64_t* rec = lds64;                                           // V coupling records
    uint16_t* tieq = reinterpret_cast<uint16_t*>(lds64 + V);         // tie queue: box index | interior << 15
    int8_t* s = reinterpret_cast<int8_t*>(tieq + ((V / 2 + 1 + 3) & ~3));  // V spins
    uint32_t* scratch = reinterpret_cast<uint32_t*>(tieq);           // set-up only: sorted site list
    __shared__ int ntie;
    __shared__ int hist[kMaxDepth], cursor[kMaxDepth];
    __shared__ int cnt_gt[2][kMaxDepth];  // sites of a colour deeper than d
    __shared__ int nsites[2];
    int8_t* cs = canon + (int64_t)r * stride;
    // exchange words: tile t owns rows_per_tile words, one per interior z-row
    const int rows_per_tile = ((L0 + tg.P[0] - 1) / tg.P[0]) * ((L1 + tg.P[1] - 1) / tg.P[1]);
    uint64_t* g0 = G0 + (int64_t)r * ntiles * rows_per_tile;
    uint64_t* g1 = G1 + (int64_t)r * ntiles * rows_per_tile;
    const uint32_t base = (uint32_t)rs[r].sweeps;

    const uint32_t mB1 = fdiv_magic((uint32_t)B[1]), mB2 = fdiv_magic((uint32_t)B[2]);
    auto gsite = [&](int b) -> int {
        const int q = (int)fdiv((uint32_t)b, mB2);
        const int z = b - q * B[2];
        const int x = (int)fdiv((uint32_t)q, mB1);
        const int y = q - x * B[1];
        return (wrapi(o[0] + x, L0) * L1 + wrapi(o[1] + y, L1)) * L2 + wrapi(o[2] + z, L2);
    };

    // ---- per-thread site lists, one per colour, deepest sites first (once)
    const int W = (B[2] + 1) >> 1;
    const int rows = B[0] * B[1];
    const uint32_t mW = fdiv_magic((uint32_t)W);
    int pk0[NS], pk1[NS];
    auto build = [&](int c, int (&pk)[NS]) {
        // enumerate the colour's box sites (row, j) -> (b, depth)
        auto site = [&](int i, int& b, int& dep) -> bool {
            const int row = (int)fdiv((uint32_t)i, mW);
            const int j = i - row * W;
            const int x = (int)fdiv((uint32_t)row, mB1);
            const int y = row - x * B[1];
            const int z = ((c - par0 - x - y) & 1) + 2 * j;
            if (z >= B[2]) return false;
            dep = kMaxDepth - 1;
            if (hk[0]) dep = min(dep, min(x, B[0] - 1 - x));
            dep = min(dep, min(y, B[1] - 1 - y));
            dep = min(dep, min(z, B[2] - 1 - z));
            b = row * B[2] + z;
            return true;
        };
        for (int d = tid; d < kMaxDepth; d += kLatThreads) {
            hist[d] = 0;
            cursor[d] = 0;
        }
        __syncthreads();
        for (int i = tid; i < rows * W; i += kLatThreads) {
            int b, dep;
            if (site(i, b, dep)) atomicAdd(&hist[dep], 1);
        }
        __syncthreads();
        if (tid == 0) {
            int acc2 = 0;
            for (int d = kMaxDepth - 1; d >= 0; --d) {
                cnt_gt[c][d] = acc2;  // sites deeper than d
                acc2 += hist[d];
            }
            nsites[c] = acc2;
        }
        __syncthreads();
        for (int i = tid; i < rows * W; i += kLatThreads) {
            int b, dep;
            if (site(i, b, dep)) {
                const int pos = cnt_gt[c][dep] + atomicAdd(&cursor[dep], 1);
                scratch[pos] = (uint32_t)(b | (dep << 20) | kSiteValid);
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < NS; ++u) {
            const int i = u * kLatThreads + tid;
            pk[u] = i < nsites[c] ? (int)scratch[i] : 0;
        }
        __syncthreads();
    };
    build(0, pk0);
    build(1, pk1);
    if (tid == 0) ntie = 0;
    // records and initial spins (internal order: colour * n/2 + g/2)
    {
        int8_t v0[NS], v1[NS];
#pragma unroll
        for (int u = 0; u < NS; ++u) {
            v0[u] = 0;
            v1[u] = 0;
            if (pk0[u] & kSiteValid) {
                const int g = gsite(site_b(pk0[u]));
                rec[site_b(pk0[u])] = Lt.rec[g];
                v0[u] = cs[g >> 1];
            }
            if (pk1[u] & kSiteValid) {
                const int g = gsite(site_b(pk1[u]));
                rec[site_b(pk1[u])] = Lt.rec[g];
                v1[u] = cs[half + (g >> 1)];
            }
        }
#pragma unroll
        for (int u = 0; u < NS; ++u) {
            if (pk0[u] & kSiteValid) s[site_b(pk0[u])] = v0[u];
            if (pk1[u] & kSiteValid) s[site_b(pk1[u])] = v1[u];
        }
    }
    __syncthreads();

    const int BZ = B[2], BYZ = B[1] * B[2];
    const int P_total = 2 * T;
    long long dE = 0;
    int nflip = 0;
    bool failed = false;

    // Moves with dE == 0 under GREEDY_TIE need an RNG draw; they are queued
    // and drawn after the pass over the colour, compacted over all lanes.
    auto phase = [&](const int (&pk)[NS], int nact) {
#pragma unroll
        for (int u = 0; u < NS; ++u) {
            if (u * kLatThreads >= nact) break;
            int p = pk[u];
            // Opaque per phase: stops the compiler from hoisting every site's
            // addresses out of the phase loop and keeping them all live.
            asm volatile("" : "+v"(p));
            if (u * kLatThreads + tid < nact) {
                const int b = site_b(p);
                const uint64_t c = rec[b];
                int f = jb(c, 6) + jb(c, 2) * s[b + BZ] + jb(c, 3) * s[b - BZ] + jb(c, 4) * s[b + 1] +
                        jb(c, 5) * s[b - 1];
                if (D == 3) f += jb(c, 0) * s[b + BYZ] + jb(c, 1) * s[b - BYZ];
                const int si = s[b];
                const int d = 2 * si * f;
                const bool inner = site_depth(p) >= k;
                if (TIE && d == 0) {
                    const int slot = atomicAdd(&ntie, 1);
                    tieq[slot] = (uint16_t)(b | ((int)inner << 15));
                }
                if (d < 0) {
                    s[b] = (int8_t)(-si);
                    if (inner) {
                        dE += d;
                        ++nflip;
                    }
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    };

    for (int e = 0; e * k < P_total; ++e) {
        const int nq = min(k, P_total - e * k);
        for (int q = 0; q < nq; ++q) {
            const int p = e * k + q;
            const uint32_t sweep = base + (uint32_t)(p >> 1);
            const int qd = min(q, kMaxDepth - 1);
            if (p & 1) phase(pk1, cnt_gt[1][qd]);
            else phase(pk0, cnt_gt[0][qd]);
            if (TIE) {
                __syncthreads();
                const int nt = ntie;
                for (int i = tid; i < nt; i += kLatThreads) {
                    const int e2 = tieq[i];
                    const int b = e2 & 0x7FFF;
                    if (rng_bit(seed, (uint32_t)gsite(b), sweep, Lt.instance_id, (uint32_t)r)) {
                        s[b] = (int8_t)(-s[b]);
                        nflip += e2 >> 15;
                    }
                }
                __syncthreads();
                if (tid == 0) ntie = 0;
            }
            __syncthreads();
        }
        // ---- exchange: publish the interior, then read the box back, every
        // word with its epoch tag.  Both passes walk contiguous z-runs (lane
        // <-> z) so a wavefront's byte accesses coalesce.  The reads write
        // only halo bytes, which the publish does not read, so no barrier
        // separates them.  After the last epoch the words are still awaited
        // (not stored): then no neighbour is still reading its box from the
        // spin array when this tile writes its interior back.
        uint64_t* gw = (e & 1) ? g1 : g0;
        const uint64_t tag = (uint64_t)(uint32_t)(e + 1) << 32;
        // one word per interior z-row: bit z set when the spin is -1
        for (int row = tid; row < nrow_int; row += kLatThreads) {
            const int x = (int)fdiv((uint32_t)row, mX1);
            const int y = row - x * X[1];
            const int b0 = ((x + hk[0]) * B[1] + (y + hk[1])) * B[2] + hk[2];
            uint32_t w = 0;
            for (int z = 0; z < X[2]; ++z) w |= (uint32_t)(s[b0 + z] < 0) << z;
            __hip_atomic_store(gw + (int64_t)tile * rows_per_tile + row, tag | w, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        const bool last = (e + 1) * k >= P_total;
        // box rows: the z-caps come from the z-neighbour tiles' rows, the
        // middle from the tile owning the row (skipped for the own interior)
        for (int row = tid; row < nrow_box && !failed; row += kLatThreads) {
            const int x = (int)fdiv((uint32_t)row, mB1);
            const int y = row - x * B[1];
            const int gx = wrapi(o[0] + x, L0), gy = wrapi(o[1] + y, L1);
            // owner of a coordinate: t = floor(((g + 1) P - 1) / L)
            const int tx = (int)(((int64_t)(gx + 1) * tg.P[0] - 1) / L0);
            const int ty = (int)(((int64_t)(gy + 1) * tg.P[1] - 1) / L1);
            const int sx = tstart(0, tx), sy = tstart(1, ty);
            const int X1t = tstart(1, ty + 1) - sy;
            const int wrow = (gx - sx) * X1t + (gy - sy);
            const int tb = (tx * tg.P[1] + ty) * tg.P[2];
            const bool inner_row = x >= hk[0] && x < hk[0] + X[0] && y >= hk[1] && y < hk[1] + X[1];
            uint64_t* al = gw + (int64_t)(tb + tzm) * rows_per_tile + wrow;
            uint64_t* ah = gw + (int64_t)(tb + tzp) * rows_per_tile + wrow;
            uint64_t* am = gw + (int64_t)(tb + tc[2]) * rows_per_tile + wrow;
            uint64_t pl = __hip_atomic_load(al, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            uint64_t ph = __hip_atomic_load(ah, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            uint64_t pm = inner_row ? tag : __hip_atomic_load(am, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // bounded wait for this epoch's words; a timeout here or in any
            // other tile raises the error flag and ends every workgroup
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
            if (failed || last) continue;
            const uint32_t wl = (uint32_t)pl, wh = (uint32_t)ph, wm = (uint32_t)pm;
            int8_t* sr = s + row * B[2];
            for (int z = 0; z < hk[2]; ++z) {
                sr[z] = (int8_t)(((wl >> (Xzm - hk[2] + z)) & 1u) ? -1 : 1);
                sr[hk[2] + X[2] + z] = (int8_t)(((wh >> z) & 1u) ? -1 : 1);
            }
            if (!inner_row)
                for (int z = 0; z < X[2]; ++z) sr[hk[2] + z] = (int8_t)(((wm >> z) & 1u) ? -1 : 1);
        }
        failed = __syncthreads_or(failed);
        if (failed) break;
    }
    // write the interior back in internal order and fold the counters
    if (!failed) {
        for (int i = tid; i < nint_all; i += kLatThreads) {
            const int row = (int)fdiv((uint32_t)i, mX2);
            const int z = i - row * X[2];
            const int x = (int)fdiv((uint32_t)row, mX1);
            const int y = row - x * X[1];
            const int b = ((x + hk[0]) * B[1] + (y + hk[1])) * B[2] + (z + hk[2]);
            const int gx = st[0] + x, gy = st[1] + y, gz = st[2] + z;
            const int g = (gx * L1 + gy) * L2 + gz;
            cs[((gx + gy + gz + Lt.c0) & 1) * half + (g >> 1)] = s[b];
        }
    }
    long long nf = nflip;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        dE += __shfl_xor(dE, off, 64);
        nf += __shfl_xor(nf, off, 64);
    }
    __shared__ long long pd[kLatWaves], pf[kLatWaves];
    if ((tid & 63) == 0) {
        pd[tid >> 6] = dE;
        pf[tid >> 6] = nf;
    }
    __syncthreads();
    if (tid == 0) {
        long long a = 0, b2 = 0;
        for (int w = 0; w < kLatWaves; ++w) {
            a += pd[w];
            b2 += pf[w];
        }
        int64_t* ap = acc + 2 * ((int64_t)r * nslots + tile);
        ap[0] += a;
        ap[1] += b2;
    }
}

// Whole lattice of replica r = blockIdx.x in one workgroup (spins in LDS,
// records read through the cache).  until_conv: stop after the first sweep
// without flips, recording lastflip as the per-phase kernels do.
template <int D, bool TIE>
__global__ __launch_bounds__(kLatThreads) void k_lattice_wg(LatticeDev Lt, int8_t* __restrict__ canon, int64_t stride,
                                                            RepState* __restrict__ rs, int64_t* __restrict__ acc,
                                                            int nslots, int T, uint64_t seed, int until_conv,
                                                            WgSolve sv, int solve)
{
    extern __shared__ uint64_t lds64[];
    int8_t* s = reinterpret_cast<int8_t*>(lds64);
    const int r = blockIdx.x;
    RepState* stp = rs + r;
    if (!solve && stp->converged) return;
    const int tid = threadIdx.x;
    const int L0 = Lt.L[0], L1 = Lt.L[1], L2 = Lt.L[2];
    const int n = Lt.n, half = n / 2;
    int8_t* cs = canon + (int64_t)r * stride;
    // load: site g <- internal index; a solve draws the random start instead
    // (the start rule of every other start kernel: the Philox bit of (site,
    // 0xFFFFFFFF, instance, restart), set meaning s = -1)
    for (int g = tid; g < n; g += kLatThreads) {
        if (solve) {
            s[g] = (int8_t)(rng_bit(seed, (uint32_t)g, 0xFFFFFFFFu, Lt.instance_id, (uint32_t)r) ? -1 : 1);
        } else {
            const int gz = g % L2, gy = (g / L2) % L1, gx = g / (L1 * L2);
            s[g] = cs[((gx + gy + gz + Lt.c0) & 1) * half + (g >> 1)];
        }
    }
    __shared__ int sweep_flips;
    if (tid == 0) sweep_flips = 0;
    __syncthreads();
    const uint32_t base = solve ? 0u : (uint32_t)stp->sweeps;
    const uint32_t mL2 = fdiv_magic((uint32_t)L2), mL1 = fdiv_magic((uint32_t)L1);
    const int hz = L2 >> 1;  // sites of one colour per z row
    long long dE = 0, nflip = 0;
    int lastflip = 0;
    for (int t = 0; t < T; ++t) {
        int my = 0;
        for (int c = 0; c < 2; ++c) {
            const int total = L0 * L1 * hz;
            for (int id = tid; id < total; id += kLatThreads) {
                const uint32_t row = fdiv((uint32_t)id, fdiv_magic((uint32_t)hz));
                const int j = id - (int)row * hz;
                const int x = (int)fdiv(row, mL1);
                const int y = (int)row - x * L1;
                const int z = ((c - Lt.c0 - x - y) & 1) + 2 * j;
                const int g = (x * L1 + y) * L2 + z;
                const uint64_t rc = Lt.rec[g];
                const int yp = y + 1 == L1 ? 0 : y + 1, ym = y == 0 ? L1 - 1 : y - 1;
                const int zp = z + 1 == L2 ? 0 : z + 1, zm = z == 0 ? L2 - 1 : z - 1;
                const int rowb = x * L1;
                int f = jb(rc, 6) + jb(rc, 2) * s[(rowb + yp) * L2 + z] + jb(rc, 3) * s[(rowb + ym) * L2 + z] +
                        jb(rc, 4) * s[(rowb + y) * L2 + zp] + jb(rc, 5) * s[(rowb + y) * L2 + zm];
                if (D == 3) {
                    const int xp = x + 1 == L0 ? 0 : x + 1, xm = x == 0 ? L0 - 1 : x - 1;
                    f += jb(rc, 0) * s[(xp * L1 + y) * L2 + z] + jb(rc, 1) * s[(xm * L1 + y) * L2 + z];
                }
                const int si = s[g];
                const int d = 2 * si * f;
                bool flip = d < 0;
                if (TIE && d == 0) flip = rng_bit(seed, (uint32_t)g, base + t, Lt.instance_id, (uint32_t)r) != 0;
                if (flip) {
                    s[g] = (int8_t)(-si);
                    dE += d;
                    ++my;
                }
            }
            __syncthreads();
        }
        (void)mL2;
        nflip += my;
        if (until_conv) {
            if (my) atomicAdd(&sweep_flips, my);
            __syncthreads();
            const int tot = sweep_flips;
            __syncthreads();
            if (tid == 0) sweep_flips = 0;
            if (tot == 0) break;
            lastflip = t + 1;
        }
    }
    // a solve ends with the exact energy of the final spins (Sec. II eq. (1)):
    // every site adds its field and its +x, +y, +z bonds, so each term counts once
    long long Efin = 0;
    for (int g = tid; g < n; g += kLatThreads) {
        const int gz = g % L2, gy = (g / L2) % L1, gx = g / (L1 * L2);
        cs[((gx + gy + gz + Lt.c0) & 1) * half + (g >> 1)] = s[g];
        if (solve) {
            const uint64_t rc = Lt.rec[g];
            const int yp = gy + 1 == L1 ? 0 : gy + 1, zp = gz + 1 == L2 ? 0 : gz + 1;
            int f = jb(rc, 6) + jb(rc, 2) * s[(gx * L1 + yp) * L2 + gz] + jb(rc, 4) * s[(gx * L1 + gy) * L2 + zp];
            if (D == 3) {
                const int xp = gx + 1 == L0 ? 0 : gx + 1;
                f += jb(rc, 0) * s[(xp * L1 + gy) * L2 + gz];
            }
            Efin -= (long long)(s[g] * f);
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        dE += __shfl_xor(dE, off, 64);
        nflip += __shfl_xor(nflip, off, 64);
        Efin += __shfl_xor(Efin, off, 64);
    }
    __shared__ long long pd[kLatWaves], pf[kLatWaves], pe[kLatWaves];
    if ((tid & 63) == 0) {
        pd[tid >> 6] = dE;
        pf[tid >> 6] = nflip;
        pe[tid >> 6] = Efin;
    }
    __syncthreads();
    if (tid == 0) {
        long long a = 0, b2 = 0, e2 = 0;
        for (int w = 0; w < kLatWaves; ++w) {
            a += pd[w];
            b2 += pf[w];
            e2 += pe[w];
        }
        if (solve) {
            // the replica's state and the call totals as a start, this run
            // and its end kernel leave them (sweeps: the first sweep without
            // a flip counts)
            int performed = T, conv = 0;
            if (until_conv && lastflip < T) {
                performed = lastflip + 1;
                conv = 1;
            }
            RepState z;
            z.E = e2;
            z.flips = b2;
            z.sweeps = performed;
            z.lastflip = until_conv ? lastflip : 0;
            z.converged = conv;
            *stp = z;
            CallStats* cs2 = sv.stats;
            atomicAdd(&cs2->attempts, (unsigned long long)((long long)performed * n));
            atomicAdd(&cs2->flips, (unsigned long long)b2);
            atomicMax(&cs2->sweeps_max, (unsigned long long)performed);
            if (until_conv && !conv) atomicAdd(&cs2->unconverged, 1ull);
        } else {
            int64_t* ap = acc + 2 * ((int64_t)r * nslots);
            ap[0] += a;
            ap[1] += b2;
            if (until_conv) stp->lastflip = lastflip;
        }
    }
    if (!solve) return;
    // the workgroup that finishes last picks the best restart (lowest energy,
    // lowest restart among equal energies) and copies the call totals out
    __shared__ int is_last;
    if (tid == 0) {
        __threadfence();
        is_last = atomicAdd(&sv.stats->done, 1ull) + 1 == sv.done_end;
    }
    __syncthreads();
    if (!is_last) return;
    __threadfence();
    const int R = (int)gridDim.x;
    long long bE = 0x7FFFFFFFFFFFFFFFll;
    int bR = 0x7FFFFFFF;
    for (int k = tid; k < R; k += kLatThreads) {  // restarts rise along a thread: the first of equal energies stays
        const long long e = __hip_atomic_load(&rs[k].E, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (e < bE) {
            bE = e;
            bR = k;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const long long e2 = __shfl_xor(bE, off, 64);
        const int r2 = __shfl_xor(bR, off, 64);
        if (e2 < bE || (e2 == bE && r2 < bR)) {
            bE = e2;
            bR = r2;
        }
    }
    __shared__ long long wE[kLatWaves];
    __shared__ int wR[kLatWaves];
    if ((tid & 63) == 0) {
        wE[tid >> 6] = bE;
        wR[tid >> 6] = bR;
    }
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < kLatWaves; ++w)
            if (wE[w] < wE[0] || (wE[w] == wE[0] && wR[w] < wR[0])) {
                wE[0] = wE[w];
                wR[0] = wR[w];
            }
        *sv.best_E = wE[0];
        *sv.best_r = wR[0];
        if (sv.stats_out) {
            CallStats c;
            c.attempts = __hip_atomic_load(&sv.stats->attempts, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            c.flips = __hip_atomic_load(&sv.stats->flips, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            c.sweeps_max = __hip_atomic_load(&sv.stats->sweeps_max, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            c.unconverged = __hip_atomic_load(&sv.stats->unconverged, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            c.done = sv.done_end;
            *sv.stats_out = c;
            // every workgroup of the solve has counted: the totals start the
            // next solve at zero
            *sv.stats = CallStats{0ull, 0ull, 0ull, 0ull, 0ull};
        }
    }
}

// ---------------------------------------------------------------------------

// Box extents of the largest tile and the per-colour site-list length per thread.
static void tile_box(const TileGeom& tg, const int L[3], int D, int B[3])
{
    for (int a = 0; a < 3; ++a) {
        const int mx = (L[a] + tg.P[a] - 1) / tg.P[a];
        B[a] = mx + ((D == 2 && a == 0) ? 0 : 2 * tg.k);
    }
}

size_t lattice_tiles_lds(const TileGeom& tg, const int L[3], int D)
{
    int B[3];
    tile_box(tg, L, D, B);
    const size_t V = (size_t)B[0] * B[1] * B[2];
    return V * 8 + ((V / 2 + 1 + 3) & ~(size_t)3) * 2 + V;
}

int64_t lattice_tiles_words(const TileGeom& tg, const int L[3])
{
    const int64_t rows = (int64_t)((L[0] + tg.P[0] - 1) / tg.P[0]) * ((L[1] + tg.P[1] - 1) / tg.P[1]);
    return rows * tg.P[0] * tg.P[1] * tg.P[2];
}

int lattice_tiles_ns(const TileGeom& tg, const int L[3], int D)
{
    int B[3];
    tile_box(tg, L, D, B);
    const long long per_colour = (long long)B[0] * B[1] * ((B[2] + 1) / 2);
    const long long ns = (per_colour + kLatThreads - 1) / kLatThreads;
    for (int c : {2, 3, 4, 5, 6, 7, 8, 10})
        if (ns <= c) return c;
    return 0;
}

template <int D, bool TIE, int NS>
static const void* tiles_kernel() { return (const void*)k_lattice_tiles<D, TIE, NS>; }

static const void* pick_tiles_kernel(int D, bool tie, int ns)
{
#define SG_NS_CASE(N)                                                                              \
    case N:                                                                                        \
        return D == 3 ? (tie ? tiles_kernel<3, true, N>() : tiles_kernel<3, false, N>())           \
                      : (tie ? tiles_kernel<2, true, N>() : tiles_kernel<2, false, N>());
    switch (ns) {
        SG_NS_CASE(2)
        SG_NS_CASE(3)
        SG_NS_CASE(4)
        SG_NS_CASE(5)
        SG_NS_CASE(6)
        SG_NS_CASE(7)
        SG_NS_CASE(8)
        SG_NS_CASE(10)
    default: return nullptr;
    }
#undef SG_NS_CASE
}

hipError_t launch_lattice_tiles(const LatticeDev& Lt, const TileGeom& tg, int8_t* canon, int64_t stride,
                                uint64_t* G0, uint64_t* G1, uint32_t* err, RepState* rs, int R,
                                int64_t* acc, int nslots, int T, uint64_t seed, int rule, hipStream_t st)
{
    const int ns = lattice_tiles_ns(tg, Lt.L, Lt.D);
    const void* kern = pick_tiles_kernel(Lt.D, rule == 1, ns);
    if (!kern) return hipErrorInvalidValue;
    const size_t lds = lattice_tiles_lds(tg, Lt.L, Lt.D);
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const int ntiles = tg.P[0] * tg.P[1] * tg.P[2];
    LatticeDev a0 = Lt;
    TileGeom a1 = tg;
    void* args[] = {&a0, &a1, &canon, &stride, &G0, &G1, &err, &rs, &acc, &nslots, &T, &seed};
    return hipLaunchCooperativeKernel(kern, dim3(ntiles * R), dim3(kLatThreads), args, (unsigned)lds, st);
}

// Co-resident workgroups of the tile kernel with this tiling, or 0 when it
// cannot launch.  A failed probe leaves no error behind for later calls.
int lattice_tiles_max_blocks(const TileGeom& tg, const int L[3], int D)
{
    const int ns = lattice_tiles_ns(tg, L, D);
    const void* kern = pick_tiles_kernel(D, true, ns);
    if (!kern) return 0;
    const size_t lds = lattice_tiles_lds(tg, L, D);
    int per_cu = 0, dev = 0, cus = 0;
    if (hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kLatThreads, lds) != hipSuccess ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return per_cu * cus;
}

hipError_t launch_lattice_wg(const LatticeDev& Lt, int8_t* canon, int64_t stride, RepState* rs, int R, int64_t* acc,
                             int nslots, int T, uint64_t seed, int rule, int until_conv, hipStream_t st,
                             const WgSolve* solve_p)
{
    const int solve = solve_p ? 1 : 0;
    const WgSolve sv = solve_p ? *solve_p : WgSolve{};
    // the LDS size is raised once per kernel variant (a call per launch costs
    // as much host time as the launch of a small lattice itself)
    static std::atomic<size_t> lds_set[4];
    const size_t lds = ((size_t)Lt.n + 7) / 8 * 8;
    const bool tie = rule == 1;
    const void* kern;
    if (Lt.D == 3) kern = tie ? (const void*)k_lattice_wg<3, true> : (const void*)k_lattice_wg<3, false>;
    else kern = tie ? (const void*)k_lattice_wg<2, true> : (const void*)k_lattice_wg<2, false>;
    std::atomic<size_t>& set = lds_set[(Lt.D == 3 ? 2 : 0) + (tie ? 1 : 0)];
    if (lds > set.load(std::memory_order_relaxed)) {
        hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        size_t cur = set.load(std::memory_order_relaxed);
        while (lds > cur && !set.compare_exchange_weak(cur, lds)) {
        }
    }
    if (Lt.D == 3) {
        if (tie)
            hipLaunchKernelGGL((k_lattice_wg<3, true>), dim3(R), dim3(kLatThreads), lds, st, Lt, canon, stride, rs, acc,
                               nslots, T, seed, until_conv, sv, solve);
        else
            hipLaunchKernelGGL((k_lattice_wg<3, false>), dim3(R), dim3(kLatThreads), lds, st, Lt, canon, stride, rs,
                               acc, nslots, T, seed, until_conv, sv, solve);
    } else {
        if (tie)
            hipLaunchKernelGGL((k_lattice_wg<2, true>), dim3(R), dim3(kLatThreads), lds, st, Lt, canon, stride, rs, acc,
                               nslots, T, seed, until_conv, sv, solve);
        else
            hipLaunchKernelGGL((k_lattice_wg<2, false>), dim3(R), dim3(kLatThreads), lds, st, Lt, canon, stride, rs,
                               acc, nslots, T, seed, until_conv, sv, solve);
    }
    return hipGetLastError();
}

}  // namespace sg
