// sg_layout.h -- packed device layout shared by the library's host code and
// its HIP kernels (internal; not part of the C-ABI).
//
// One instance is stored colour-major: spins are relabelled so that each
// colour class occupies a contiguous range of internal indices, and inside a
// class spins are ordered by decreasing incidence count (stable, so equal
// counts keep increasing external index).  Couplings are stored in sliced
// ELLPACK form with slices of 64 rows, one row per lane of a wavefront: the
// k-th coupling of the row in lane l of a slice sits at
// ebase + k*64 + l, so one coupling step of a wavefront reads 256
// contiguous bytes.  Each coupling is one 32-bit word (partner << 8 | J & 255)
// with the partner's internal index in the top 24 bits and J as int8 in the
// low byte.  A 3-spin hyper-coupling (i, a, b; K) is stored in the row of
// each of its three members as two words (a << 8 | K & 255) and b.  Padding
// words are zero (partner 0, coefficient 0) and contribute nothing.
#pragma once
#include <stdint.h>

namespace sg {

constexpr int kSlice = 64;        // rows per slice (one wavefront)
constexpr int kPhaseWaves = 4;    // wavefronts per block of the phase kernels
constexpr int kPhaseThreads = kSlice * kPhaseWaves;

struct Slice {          // 16 bytes
    uint32_t row0;      // internal index of the spin in lane 0
    uint32_t ebase;     // word offset of the slice's first coupling
    uint32_t tbase;     // word offset of the slice's first hyper-coupling
    uint16_t ew;        // coupling words per row in this slice
    uint8_t tw;         // hyper-couplings per row in this slice
    uint8_t rows;       // valid rows (1..64)
};
static_assert(sizeof(Slice) == 16, "Slice must be 16 bytes");

// Device view of one instance (pointers into the caller's workspace).
struct InstDev {
    const uint32_t* nbr;     // coupling words
    const uint32_t* ta;      // hyper-coupling words (a << 8 | K)
    const uint32_t* tb;      // hyper-coupling partner b
    const int8_t* h;         // field per internal index
    const uint32_t* ext;     // internal -> external index (RNG counter word 0)
    const Slice* slices;     // all slices, colour by colour
    int32_t n;
    int32_t nslices;
    uint32_t instance_id;
    int32_t has_tri;
};

// Wide form of an instance whose values or sizes exceed the packed words:
// couplings, fields or hyper-couplings outside int8 (any int32 value, with
// |h_i| + sum|J_ij| + sum|K| < 2^31 per spin), more than 2^24 - 1 spins, more
// than 255 hyper-couplings on one spin or 65535 couplings on one row, or more
// restarts than one launch dimension holds.  Same colour-major relabel and
// sliced rows as the packed form; the partner index and the coefficient sit
// in separate 32-bit words at the same sliced position (k-th entry of the row
// in lane l at base + k*64 + l).
struct WSlice {          // 32 bytes
    uint64_t ebase;      // word offset of the slice's first coupling
    uint64_t tbase;      // word offset of the slice's first hyper-coupling
    uint32_t row0;       // internal index of the spin in lane 0
    uint32_t ew;         // couplings per row in this slice
    uint32_t tw;         // hyper-couplings per row in this slice
    uint32_t rows;       // valid rows (1..64)
};
static_assert(sizeof(WSlice) == 32, "WSlice must be 32 bytes");

struct WideDev {
    const uint32_t* nbr;     // coupling partner (internal index)
    const int32_t* J;        // coupling value
    const uint32_t* ta;      // hyper-coupling partners a and b
    const uint32_t* tb;
    const int32_t* K;        // hyper-coupling value
    const int32_t* h;        // field per internal index
    const uint32_t* ext;     // internal -> external index (RNG counter word 0)
    const WSlice* slices;    // all slices, colour by colour
    int32_t n;
    int32_t nslices;
    uint32_t instance_id;
    int32_t has_tri;
};

// Per-replica state, 32 bytes.
struct RepState {
    int64_t E;          // tracked energy
    int64_t flips;      // moves applied since the start
    int64_t sweeps;     // sweeps performed since the start (absolute sweep index of the next sweep)
    int32_t lastflip;   // within a call: 1 + relative index of the last sweep that flipped
    int32_t converged;  // 1 once a sweep flipped nothing under until_converged
};
static_assert(sizeof(RepState) == 32, "RepState must be 32 bytes");

// Per-call totals written by the end-of-call kernel.
struct CallStats {
    unsigned long long attempts;
    unsigned long long flips;
    unsigned long long sweeps_max;
    unsigned long long unconverged;
    unsigned long long done;  // workgroups finished (the one-launch solve of small lattices)
};

// Lattice (implicit neighbour) layout for the LDS tile schedules.  Sites are
// (x, y, z), z fastest; 2-D lattices use L[0] = 1.  One 64-bit record per
// site: bytes 0..5 = J to the +x, -x, +y, -y, +z, -z neighbour, byte 6 = h.
struct LatticeDev {
    const uint64_t* rec;     // n records, site order
    int32_t L[3];
    int32_t D;               // 2 or 3
    int32_t c0;              // colour of site 0
    int32_t n;
    uint32_t instance_id;
};

struct TileGeom {
    int32_t P[3];            // tiles per axis
    int32_t k;               // colour phases per halo exchange (= halo width)
};

// Device table entry of one instance for the batched schedules.
struct InstTab {
    InstDev I;
    int8_t* spins;           // replica 0's spins (internal order)
    int64_t spin_stride;     // bytes between replicas
    int64_t rep_base;        // index of replica 0 in the handle's replica array
    int32_t C;               // colours
    int32_t ctab_off;        // offset of the instance's C+1 colour slice starts in the colour table
    int32_t nbr_words;       // coupling words of the sliced layout
    int32_t tri_words;       // hyper-coupling words (each of ta, tb)
    // energy terms of an instance of at most 2048 spins, each at its smallest
    // internal index i: n_eh fields (i | h << 22), then n_ee couplings
    // (i | j << 11 | J << 22), then n_et hyper-couplings as word pairs
    // (i | a << 11 | K << 22, b); coefficients as 8-bit two's complement
    const uint32_t* eterm;
    int32_t n_eh, n_ee, n_et, eterm_pad;
    // Per-spin term rows in external order for the lane-per-replica pass
    // kernel (null when the instance does not qualify; layout in
    // sg_fm_lanes.hip): fml_dc coupling words and fml_tt hyper-couplings per
    // spin.
    const uint32_t* fml;
    int32_t fml_dc, fml_tt;
};

// Per-spin term rows in external order for the pass kernel of instances
// beyond 4096 spins (sg_fm_big.hip): spin e's row is the stride words from
// rows + e * stride, unused entries zero.  Packed form (wide = 0): a word
// with the field in its low byte (int8), dc coupling words (partner << 8 |
// J & 255), tt hyper-coupling pairs (a << 8 | K & 255, b).  Wide form: the
// field (int32), dc pairs (partner, J), tt triples (a, b, K).
struct FmbRows {
    const uint32_t* rows;
    int32_t stride, dc, tt, wide;
};

struct BlockItem {           // k_block: restarts [r0, r0 + nr) of instance inst
    int32_t inst;
    int32_t r0;
    int32_t nr;
    int32_t pad;
};

struct StartUnit {           // batched start / energy: a range of replica g
    int64_t g;               // replica (handle order)
    int32_t inst;            // its instance
    int32_t off;             // first spin (start) or first slice (energy)
};

struct EnergySeg {           // batched energy: the units of replica g
    int64_t g;               // replica (handle order)
    int64_t u0;              // its first energy unit
    int32_t nu;              // its number of energy units
    int32_t pad;
};

struct QueueItem {           // k_queue: restart r of instance inst
    int32_t inst;
    int32_t r;
};

// Dense hyper-Ising instance (at most 64 spins, couplings over any set of
// spins, int64 coefficients): terms by spin (the other members and the
// coefficient of every term holding spin i, entries dstart[i] .. dstart[i+1]),
// the whole term list, and the sweep order (colours ascending, spins of a
// colour ascending).  Energy E = -sum_t coef_t prod_{i in t} s_i.
struct DenseTab {
    const int32_t* dstart;   // n + 1
    const uint64_t* dmask;   // other members of the term
    const int64_t* dcoef;
    const uint64_t* tmask;   // every term once
    const int64_t* tcoef;
    const int32_t* order;    // n spins in sweep order
    int8_t* spins;           // replica 0, +-1 per spin
    int64_t spin_stride;
    int64_t rep_base;
    int32_t n;
    int32_t nterms;
    uint32_t instance_id;
    int32_t pad;
};

}  // namespace sg
