// sg_host.cpp -- host core and C-ABI of the spin-glass local-search library.
//
// Instance ingest (validation, colouring, colour-major relabel, sliced
// coupling layout, workspace layout), the run driver that enqueues the HIP
// kernels of sg_kernels.hip on the caller's stream, and readout.  The
// semantics of every entry point are documented in include/sg.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <numeric>
#include <string>
#include <atomic>
#include <thread>
#include <vector>

#include "sg.h"
#include "sg_launch.h"
#include "sg_layout.h"

namespace {

thread_local std::string g_err;

sg_status fail(sg_status code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

sg_status hip_fail(hipError_t e, const char* what)
{
    return fail(SG_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define SG_HIP(call, what)                                   \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return hip_fail(e_, what);     \
    } while (0)

constexpr uint64_t kAlign = 256;
inline uint64_t align_up(uint64_t v, uint64_t a = kAlign) { return (v + a - 1) / a * a; }

// f(lo, hi) over [0, count) in contiguous ranges on up to kHostThreads host
// threads (one below 2^16 items): the per-row loops of a large instance's
// ingest.  A range starting at lo may keep per-range results in slot
// lo * kHostThreads / count: distinct and increasing over the ranges.
constexpr unsigned kHostThreads = 4;
template <class F>
void parallel_ranges(int64_t count, F&& f)
{
    unsigned T = std::thread::hardware_concurrency();
    T = std::min(T ? T : 1u, kHostThreads);
    if (count < 65536 || T <= 1) {
        f((int64_t)0, count);
        return;
    }
    const int64_t step = (count + T - 1) / T;
    std::vector<std::thread> th;
    for (unsigned t = 1; t < T; ++t) {
        const int64_t lo = std::min<int64_t>(count, (int64_t)t * step), hi = std::min<int64_t>(count, lo + step);
        if (lo < hi) th.emplace_back([&f, lo, hi] { f(lo, hi); });
    }
    f((int64_t)0, std::min<int64_t>(count, step));
    for (std::thread& x : th) x.join();
}

constexpr int32_t kMaxN = (1 << 24) - 1;
constexpr int32_t kMaxCoef = 127;
constexpr int64_t kMaxField = (1 << 23) - 1;
constexpr int32_t kMaxRestarts = 65535;         // packed form: restarts within one launch dimension
constexpr int32_t kMaxWideN = 1 << 30;          // wide form: spins per instance
constexpr int64_t kMaxWideField = INT32_MAX;    // per-spin |h| + sum|J| + sum|K| (int32 field)
constexpr int32_t kMaxLatticeTiles = 1024;
constexpr int32_t kConvChunk = 16384;  // sweeps per bit-plane launch under the stopping rule (counter slots)
constexpr size_t kLatLdsBudget = 160 * 1024 - 4 * 1024;  // dynamic LDS of the tile kernels
constexpr int32_t kFmMaxN = 4096;          // largest instance of the pass-based search (LDS per wavefront)
constexpr int32_t kFmlMaxN = 1024;         // one replica per lane: instances up to this size ...
constexpr int64_t kFmlMaxW = 127;          // ... whose per-spin sum of |coefficients| fits a byte gain
constexpr int32_t kLaneStartMaxN = 2048;       // lane-per-replica start/energy: instances up to this size ...
constexpr int32_t kLaneStartMinR = 32;         // ... with at least this many restarts, ...
constexpr int64_t kLaneStartMinTotal = 16384;  // ... when such replicas fill the chip (64 per wavefront)  // instances below this size start and evaluate in batched launches

struct HostInst {
    int32_t n = 0;
    int64_t m = 0, t = 0;
    int32_t C = 0;
    uint32_t id = 0;
    int32_t R = 1;
    int32_t lattice = 0;
    int32_t dims[3] = {0, 0, 0};
    std::vector<int32_t> colour;       // external order
    std::vector<uint32_t> ext_of;      // internal -> external
    std::vector<int32_t> colour_slice; // C+1 slice offsets
    std::vector<sg::Slice> slices;
    std::vector<uint32_t> nbr, ta, tb;
    std::vector<int8_t> h;             // internal order
    std::vector<uint32_t> eterm;       // energy terms (instances of at most 2048 spins)
    int32_t n_eh = 0, n_ee = 0, n_et = 0;
    int32_t nslots = 1;                // phase-kernel blocks per colour (max over colours)
    int32_t acc_slots = 1;             // accumulator slots per replica (max over schedules)
    int64_t rep_base = 0;
    // lattice schedule (implicit neighbours)
    int32_t lat_ok = 0;                // lattice hint accepted, even extents, checkerboard colouring
    uint64_t off_fmb_rows = UINT64_MAX;  // term rows in external order for the large-instance pass kernel
    int32_t fmb_dc = 0, fmb_tt = 0;      // their coupling and hyper-coupling widths
    int32_t lat_msc = 0;               // every lattice bond is +-1 and |h| <= 2 (bit-plane kernel)
    int64_t max_w = 0;                 // largest sum of |coefficients| over one spin's terms
    uint64_t fml_off = UINT64_MAX;     // word offset of its per-spin term rows (lane pass kernel), or none
    int32_t fml_dc = 0, fml_tt = 0;    // coupling words / hyper-couplings per row
    int32_t bits_ok = 0;               // at most 2048 spins, every |coefficient| <= 15 and per spin
                                       // sum |c| <= 255 (bit-sliced block kernel)
    // last tiling decision and the settings it was made for (rule, knobs)
    mutable std::array<int32_t, 6> tile_key{{-1, -1, -1, -1, -1, -1}};
    mutable sg::TileGeom tile_geom{};
    mutable int32_t tile_msc = 0;
    mutable int32_t tile_found = 0;
    mutable double tile_model_phase_us = 0.0, tile_model_ex_us = 0.0;  // cost model of the bit-plane tiling
    int32_t lat_L[3] = {0, 0, 0};      // (x, y, z) extents, z fastest; 2-D: (1, Lx, Ly)
    int32_t lat_D = 0;
    int32_t lat_c0 = 0;
    std::vector<uint64_t> lat_rec;     // per-site coupling record
    uint64_t off_lat_rec = 0, off_lat_g = 0, lat_g_bytes = 0;
    uint64_t off_lat_cnt = 0;          // per-sweep tile counters of the bit-plane kernel's stopping rule
    // workspace offsets (bytes)
    uint64_t off_nbr = 0, off_ta = 0, off_tb = 0, off_h = 0, off_ext = 0, off_slices = 0, off_eterm = 0;
    uint64_t off_spins = 0, spin_stride = 0, off_acc = 0;
    uint64_t off_fields = 0, field_stride = 0;  // maintained local fields (ints per replica), when enabled
    // wide form (values or sizes beyond the packed words, sg_layout.h)
    int32_t wide = 0;
    std::vector<uint32_t> w_nbr, w_ta, w_tb;
    std::vector<int32_t> w_J, w_K, w_h;
    std::vector<sg::WSlice> w_slices;
    uint64_t off_wnbr = 0, off_wJ = 0, off_wta = 0, off_wtb = 0, off_wK = 0, off_wh = 0, off_wslices = 0;
    // dense hyper-Ising instance (sg_load_dense)
    int32_t dense = 0;
    std::vector<int32_t> d_start, d_order;
    std::vector<uint64_t> d_mask, t_mask;
    std::vector<int64_t> d_coef, t_coef;
    uint64_t off_dstart = 0, off_dmask = 0, off_dcoef = 0, off_tmask = 0, off_tcoef = 0, off_dorder = 0;
};

}  // namespace

struct sg_ctx {
    std::vector<HostInst> insts;
    int64_t total_reps = 0;
    uint64_t bytes = 0;
    uint64_t off_reps = 0, off_stats = 0, off_flag = 0, off_eout = 0, off_slots = 0;
    uint64_t off_best_E = 0, off_best_r = 0, off_rep_base = 0, off_restarts = 0, off_err = 0, off_solve = 0;
    // tuning knobs (sg_tune)
    int32_t lattice_k = 4;             // phases per halo exchange of the lattice tile schedule
    int32_t lattice_max_tiles = 0;     // 0 = as many as fit co-resident
    int32_t lattice_wg_max_n = 150000; // largest lattice run as one workgroup per replica
    int32_t block_rg = 0;              // restarts per block workgroup (0 = largest that fits)
    int32_t block_min_restarts = 32;   // AUTO uses the block schedule from this many restarts
    int32_t block_groups = 0;          // restart groups per block workgroup (0 = auto, up to 4)
    int32_t block_bits = 1;            // GREEDY block schedule in bit-sliced form where it applies
    int32_t bits_groups = 8;           // most groups of 32 restarts per bit-sliced workgroup (2, 4, 8, 16)
    int32_t fm_key32 = 1;              // FM moves chosen on 32-bit keys where the gains allow
    int32_t fm_waves = 0;              // most wavefronts per FM workgroup (0 = 16); the most resident are taken
    int32_t last_fm_waves = 0;         // what the last FM call used
    std::array<int64_t, 5> fm_key{{-1, -1, -1, -1, -1}};  // setting of the cached FM workgroup size
    int32_t fm_waves_cached = 0;
    int32_t fml_ws = 1;                // workspace holds the per-spin term lists of the lane pass kernel
    int32_t fm_lanes = 1;              // FM runs one replica per lane where the instance allows
    int32_t fm_lane_restarts = 0;      // restarts per lane-kernel item (0 = chosen to fill the device)
    // the pass-based search on instances beyond a wavefront's LDS: replicas
    // run at once (0: none; its scratch is part of the workspace), the largest
    // such instance, and the workspace areas
    int32_t fm_slots = 0;
    int32_t fmb_nmax = 0;
    int64_t fmb_reps = 0, fmb_slot_spins = 0, fmb_slot_leaves = 0;
    uint64_t off_fmb_half = 0, off_fmb_moves = 0, off_fmb_leaf = 0, off_fmb_spin = 0, off_fmb_ptr = 0,
             off_fmb_items = 0, off_fmb_cnt = 0;
    int32_t last_fm_big = 0;           // replicas of the last FM call run on that kernel
    int32_t fm_lane_waves = 0;         // wavefronts per lane-kernel workgroup sharing an item (0 = 1)
    int32_t last_fm_lanes = 0;         // replicas of the last FM call run one per lane
    int32_t last_fm_lane_nr = 0;       // restarts per item of that call
    std::vector<uint32_t> h_fml;       // term lists of every qualifying instance
    uint64_t off_fml = 0, off_fmitems = 0;
    int64_t fm_item_cap = 0;
    std::vector<sg::BlockItem> h_fmitems;
    int32_t defer_energy = 1;          // a drawn start whose run computes final energies gets its energy later
    int32_t last_key32 = 0;            // the last FM call used 32-bit keys
    int32_t queue_wave_max_n = 512;    // queue items up to this size run one per wavefront (fastest measured)
    int32_t queue_grid = 0;            // persistent queue grid (0 = co-resident capacity)
    int32_t queue_min_items = 32;      // AUTO uses the queue schedule from this many items
    int32_t graph_sweeps = 32;         // sweeps per captured graph (SG_SCHED_GRAPH)
    int32_t auto_graph = 0;            // SG_SCHED_AUTO records per-phase launches in graphs (SG_SCHED_GRAPH)
    int32_t conv_chunk = kConvChunk;   // sweeps per bit-plane launch under the stopping rule
    int32_t lattice_msc = 1;           // use the bit-plane tile kernel where it applies
    int32_t msc_k = 0;                 // its halo width (0 = chosen by the cost model)
    int32_t last_msc = 0;              // the last tile launch used the bit-plane kernel
    int32_t last_bits = 0;             // the last block-schedule call used the bit-sliced kernel
    int32_t fields_ws = 0;             // workspace holds local fields per replica (SG_SCHED_FIELDS)
    int32_t dense = 0;                 // a handle of dense hyper-Ising instances
    uint64_t off_dtab = 0, off_ditems = 0;
    std::vector<sg::BlockItem> h_ditems;  // (instance, first restart, count <= 64)
    int32_t dense_nmax = 1;
    hipStream_t cap_stream = nullptr;  // private stream used only to record graphs
    uint64_t off_tbase = 0;            // one sweep base per instance (graph replays)
    uint64_t off_tab = 0, off_ctab = 0, off_bitems = 0, off_qitems = 0, off_qcnt = 0;
    uint64_t off_rep_inst = 0;
    // batched start / energy of the replicas not started one lane each: units
    // of 1024 spins (start) and of four slices (energy)
    std::vector<sg::StartUnit> h_sunits, h_eunits;
    std::vector<sg::EnergySeg> h_esegs;  // the energy units of each replica
    uint64_t off_sunits = 0, off_eunits = 0, off_esegs = 0, off_eparts = 0;
    std::vector<sg::BlockItem> h_litems;       // lane-per-replica start items (instance, r0, count <= 64)
    int32_t lane_nmax = 1;
    uint64_t off_litems = 0;
    bool lanes_on = false;
    int64_t n_block_item_cap = 0, ctab_len = 0;
    std::vector<sg::BlockItem> h_bitems;
    std::vector<sg::QueueItem> h_qitems;
    uint8_t* dev = nullptr;
    hipStream_t stream = nullptr;
    bool bound = false;
    std::vector<uint8_t> started;
    // Start energies left out by sg_init_spins: e_deferred marks the instances
    // (1: lane start, the bit-sliced kernel writes the energies; 2: unit start,
    // the queue kernel writes them at convergence), e_pending is set until a
    // run has written them or an energy pass has computed them.
    std::vector<uint8_t> e_deferred;
    bool e_pending = false;
    std::vector<uint8_t> e_written;  // this call's kernels wrote the final energies of the instance
    bool lat_err_check = false;  // the current call launched tile kernels: read their error flag at its end
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipEvent_t evh0 = nullptr, evh1 = nullptr;  // around the hot kernel(s) of the last schedule run
    // pinned host memory for the small results a call reads back (sg_bind;
    // none after sg_bind_noalloc, whose callers cannot allocate): a copy into
    // pageable memory waits for the device, one into pinned memory does not,
    // so the copies of one call share its single synchronisation
    uint8_t* pin = nullptr;
    // the call totals are zero: the last sg_solve in one launch per instance
    // left them so (its last workgroup clears them), and no run has used them since
    bool stats_zero = false;
    double hot_us = 0.0;                        // their device time, microseconds
    int32_t hot_launches = 0;                   // launches inside that interval
    int32_t last_tiles[4] = {0, 0, 0, 0};  // tiling of the last lattice tile launch
    // latency model of the last bit-plane launch: mean colour phase and exchange
    // cost (microseconds), and how many of each the launch holds
    double last_model_phase_us = 0.0, last_model_ex_us = 0.0;
    int64_t last_model_phases = 0, last_model_exchanges = 0;
    int32_t last_queue_grid = 0;

    template <class T>
    T* at(uint64_t off) const { return reinterpret_cast<T*>(dev + off); }

    sg::InstDev view(const HostInst& q) const
    {
        sg::InstDev I;
        I.nbr = at<uint32_t>(q.off_nbr);
        I.ta = at<uint32_t>(q.off_ta);
        I.tb = at<uint32_t>(q.off_tb);
        I.h = at<int8_t>(q.off_h);
        I.ext = at<uint32_t>(q.off_ext);
        I.slices = at<sg::Slice>(q.off_slices);
        I.n = q.n;
        I.nslices = (int32_t)q.slices.size();  // 0 for a wide instance: no packed kernel walks it
        I.instance_id = q.id;
        I.has_tri = q.t > 0 ? 1 : 0;
        return I;
    }
    sg::WideDev wview(const HostInst& q) const
    {
        sg::WideDev I;
        I.nbr = at<uint32_t>(q.off_wnbr);
        I.J = at<int32_t>(q.off_wJ);
        I.ta = at<uint32_t>(q.off_wta);
        I.tb = at<uint32_t>(q.off_wtb);
        I.K = at<int32_t>(q.off_wK);
        I.h = at<int32_t>(q.off_wh);
        I.ext = at<uint32_t>(q.off_ext);
        I.slices = at<sg::WSlice>(q.off_wslices);
        I.n = q.n;
        I.nslices = (int32_t)q.w_slices.size();
        I.instance_id = q.id;
        I.has_tri = q.t > 0 ? 1 : 0;
        return I;
    }
    sg::RepState* reps() const { return at<sg::RepState>(off_reps); }

    sg::LatticeDev lat_view(const HostInst& q) const
    {
        sg::LatticeDev L;
        L.rec = at<uint64_t>(q.off_lat_rec);
        for (int a = 0; a < 3; ++a) L.L[a] = q.lat_L[a];
        L.D = q.lat_D;
        L.c0 = q.lat_c0;
        L.n = q.n;
        L.instance_id = q.id;
        return L;
    }
};

namespace {

// ---------------------------------------------------------------------------
// ingest

// A host array that keeps its memory from one use to the next and is left
// uninitialised when it grows: the large temporaries of an ingest reuse the
// pages of the same thread's previous ingest instead of faulting in fresh
// ones, and the threads that fill a grown array touch its pages in parallel.
template <class T>
struct Scratch {
    std::unique_ptr<T[]> p;
    size_t cap = 0;
    T* get(size_t count)
    {
        if (count > cap) {
            p.reset(new T[count]);
            cap = count;
        }
        return p.get();
    }
};

// Every term of an instance at each of its spins, grouped by spin (external
// index) in input order, edges before triples: entry q of spin i (start[i] <=
// q < start[i + 1]) names the term's other spin a[q] and, for a triple, its
// third spin b[q] (-1 for an edge), with the term's coefficient c[q].  This is
// the primal adjacency the colouring reads, and the source of the per-spin
// sums, the duplicate check and the incidence lists.
struct IncTerm {
    int32_t a, b, c;
};
struct Incidence {
    const int64_t* start = nullptr;
    const IncTerm* e = nullptr;
};

struct IncEntry {
    int32_t row, a, b, c;
};

// One thread's ingest temporaries (the arrays behind Incidence among them:
// valid until that thread's next ingest).
struct IngestScratch {
    Scratch<int64_t> start, es, ts;
    Scratch<int32_t> deg, tdeg;
    Scratch<IncTerm> terms;
    Scratch<IncEntry> bucket;
    Scratch<uint32_t> ew, twa, twb, tmp, int_of;
};

IngestScratch& ingest_scratch()
{
    thread_local IngestScratch s;
    return s;
}

// Builds the incidences of an instance whose spin indices are all in range,
// on up to kHostThreads threads: each thread sorts the incidences of its
// range of terms into buckets by range of spins, then each thread gathers
// the bucket of its spins in term order (so the result does not depend on
// the thread count).
void build_incidence(const sg_instance_desc& d, Incidence& I)
{
    const int64_t n = d.n, m = d.m, t = d.t, terms = m + t;
    unsigned T = std::thread::hardware_concurrency();
    T = std::min(T ? T : 1u, kHostThreads);
    if (terms < 65536) T = 1;
    // range r holds the spins i with i * T / n == r: [lo(r), lo(r + 1))
    auto dest = [&](int64_t row) { return (size_t)(row * (int64_t)T / n); };
    auto lo = [&](int64_t r) { return (n * r + (int64_t)T - 1) / (int64_t)T; };
    // the incidences of term k: (spin, other, third, coefficient)
    auto visit = [&](int64_t k, auto&& out) {
        if (k < m) {
            const int32_t x = d.ei[k], y = d.ej[k];
            out(x, y, -1, d.J[k]);
            out(y, x, -1, d.J[k]);
        } else {
            const int64_t u = k - m;
            const int32_t x = d.tri[3 * u], y = d.tri[3 * u + 1], z = d.tri[3 * u + 2];
            out(x, y, z, d.K[u]);
            out(y, x, z, d.K[u]);
            out(z, x, y, d.K[u]);
        }
    };
    auto run = [&](auto&& body) {
        std::vector<std::thread> th;
        for (unsigned x = 1; x < T; ++x) th.emplace_back([&body, x] { body(x); });
        body(0u);
        for (std::thread& y : th) y.join();
    };
    auto chunk = [&](unsigned sidx, int64_t& k0, int64_t& k1) {
        k0 = terms * sidx / T;
        k1 = terms * (sidx + 1) / T;
    };
    std::vector<std::vector<int64_t>> at(T, std::vector<int64_t>(T, 0));
    run([&](unsigned sidx) {
        int64_t k0, k1;
        chunk(sidx, k0, k1);
        std::vector<int64_t>& c = at[sidx];
        for (int64_t k = k0; k < k1; ++k) visit(k, [&](int32_t row, int32_t, int32_t, int32_t) { c[dest(row)]++; });
    });
    // bucket r (entries base[r] .. base[r + 1] - 1): the entries of term
    // ranges 0, 1, ... in turn
    IngestScratch& S = ingest_scratch();
    std::vector<int64_t> base(T + 1, 0);
    for (unsigned r = 0; r < T; ++r) {
        int64_t size = 0;
        for (unsigned x = 0; x < T; ++x) {
            const int64_t c = at[x][r];
            at[x][r] = base[r] + size;
            size += c;
        }
        base[r + 1] = base[r] + size;
    }
    IncEntry* bucket = S.bucket.get(std::max<size_t>((size_t)base[T], 1));
    run([&](unsigned sidx) {
        int64_t k0, k1;
        chunk(sidx, k0, k1);
        std::vector<int64_t>& o = at[sidx];
        for (int64_t k = k0; k < k1; ++k)
            visit(k, [&](int32_t row, int32_t a, int32_t b, int32_t c) {
                const size_t r = dest(row);
                bucket[(size_t)o[r]++] = IncEntry{row, a, b, c};
            });
    });
    // per range: its spins' counts, offsets (its entries start at base[r]),
    // then its entries in bucket order
    const size_t total = std::max<size_t>((size_t)base[T], 1);
    int64_t* start = S.start.get((size_t)n + 1);
    IncTerm* E = S.terms.get(total);
    run([&](unsigned r) {
        const int64_t r0 = lo(r), r1 = lo(r + 1);
        for (int64_t i = r0; i < r1; ++i) start[i + 1] = 0;
        if (r == 0) start[0] = 0;
        for (int64_t k = base[r]; k < base[r + 1]; ++k) start[bucket[k].row + 1]++;
        int64_t acc = base[r];
        for (int64_t i = r0; i < r1; ++i) {
            const int64_t c = start[i + 1];
            start[i + 1] = acc;  // fill position of spin i, then its end
            acc += c;
        }
        for (int64_t k = base[r]; k < base[r + 1]; ++k) {
            const IncEntry& e = bucket[k];
            E[start[e.row + 1]++] = IncTerm{e.a, e.b, e.c};
        }
    });
    I.start = start;
    I.e = E;
}

// First-fit: spin i takes the smallest colour unused by primal neighbours j < i.
int32_t first_fit(const Incidence& P, int32_t n, std::vector<int32_t>& colour)
{
    colour.assign((size_t)n, 0);
    std::vector<int32_t> seen;  // seen[c] == i + 1 when colour c is taken by a lower neighbour of i
    int32_t ncol = 0;
    auto mark = [&](int32_t j, int32_t i) {
        if (j < 0 || j >= i) return;
        const int32_t c = colour[j];
        if ((size_t)c >= seen.size()) seen.resize((size_t)c + 1, 0);
        seen[c] = i + 1;
    };
    for (int32_t i = 0; i < n; ++i) {
        for (int64_t q = P.start[i]; q < P.start[i + 1]; ++q) {
            mark(P.e[q].a, i);
            mark(P.e[q].b, i);
        }
        int32_t c = 0;
        while ((size_t)c < seen.size() && seen[c] == i + 1) ++c;
        colour[i] = c;
        ncol = std::max(ncol, c + 1);
    }
    return ncol;
}

// Device-to-host copies of one call.  A copy of at most kPinBytes in total
// goes through the handle's pinned buffer and reaches its destination in
// finish(), after the call's stream synchronisation; a larger one, or any
// copy of a handle without the buffer, goes straight to its destination.
constexpr size_t kPinBytes = 64 * 1024;

class CopiesOut {
  public:
    explicit CopiesOut(const sg_ctx* H) : pin_(H->pin) {}
    hipError_t copy(void* dst, const void* src, size_t bytes, hipStream_t st)
    {
        if (pin_ && used_ + bytes <= kPinBytes) {
            const hipError_t e = hipMemcpyAsync(pin_ + used_, src, bytes, hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) pend_.push_back({dst, used_, bytes});
            used_ += (bytes + 15) & ~(size_t)15;
            return e;
        }
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st);
    }
    // only after the stream has been synchronised
    void finish()
    {
        for (const Pending& c : pend_) std::memcpy(c.dst, pin_ + c.off, c.bytes);
        pend_.clear();
        used_ = 0;
    }

  private:
    struct Pending {
        void* dst;
        size_t off, bytes;
    };
    uint8_t* pin_;
    size_t used_ = 0;
    std::vector<Pending> pend_;
};

// Checks an instance.  *wide (when given) is set when its values or sizes
// exceed the packed words (int8 coefficients, 24-bit spin index, per-spin
// |h| + sum|J| + sum|K| < 2^23, restarts within one launch dimension): such
// an instance is stored in the wide form.  SG_ERANGE only when a spin's
// |h_i| + sum|J_ij| + sum|K| exceeds 2^31 - 1 (its field would not fit int32),
// when sum|J| + sum|h| + sum|K| exceeds 2^63 - 1 (an energy would not fit
// int64), or when n exceeds 2^30 (index arithmetic).
sg_status validate(const sg_instance_desc& d, int idx, bool* wide = nullptr, Incidence* inc = nullptr)
{
    bool w = false;
    if (d.n < 1) return fail(SG_EINVAL, "instance %d: n must be >= 1", idx);
    if (d.n > kMaxWideN) return fail(SG_ERANGE, "instance %d: n = %d exceeds %d", idx, d.n, kMaxWideN);
    if (d.n > kMaxN) w = true;
    if (d.m < 0 || d.t < 0) return fail(SG_EINVAL, "instance %d: negative edge or triple count", idx);
    if (d.m > 0 && (!d.ei || !d.ej || !d.J)) return fail(SG_EINVAL, "instance %d: edge arrays missing", idx);
    if (d.t > 0 && (!d.tri || !d.K)) return fail(SG_EINVAL, "instance %d: triple arrays missing", idx);
    if (d.restarts < 1) return fail(SG_EINVAL, "instance %d: restarts must be >= 1", idx);
    if (d.restarts > kMaxRestarts) w = true;
    const int64_t n = d.n;
    __int128 total = 0;  // sum |J| + sum |h| + sum |K|
    {
        // indices, self-loops, coefficient sizes and the total, by ranges of edges
        std::vector<int64_t> bad_at(kHostThreads, -1);
        std::vector<__int128> part(kHostThreads, 0);
        std::vector<char> big(kHostThreads, 0);
        parallel_ranges(d.m, [&](int64_t k0, int64_t k1) {
            const size_t slot = (size_t)(k0 * kHostThreads / std::max<int64_t>(d.m, 1));
            __int128 sum = 0;
            bool b8 = false;
            for (int64_t k = k0; k < k1; ++k) {
                const int64_t a = d.ei[k], b = d.ej[k];
                if (a < 0 || a >= n || b < 0 || b >= n || a == b) {
                    bad_at[slot] = k;
                    return;
                }
                const int64_t c = std::llabs((int64_t)d.J[k]);
                b8 = b8 || c > kMaxCoef;
                sum += c;
            }
            part[slot] = sum;
            big[slot] = b8;
        });
        for (size_t t = 0; t < bad_at.size(); ++t)
            if (bad_at[t] >= 0) {
                const int64_t k = bad_at[t], a = d.ei[k], b = d.ej[k];
                if (a < 0 || a >= n || b < 0 || b >= n)
                    return fail(SG_EINVAL, "instance %d: edge %lld has a spin index out of range", idx, (long long)k);
                return fail(SG_EINVAL, "instance %d: edge %lld is a self-loop on spin %lld", idx, (long long)k,
                            (long long)a);
            }
        for (size_t t = 0; t < part.size(); ++t) {
            total += part[t];
            w = w || big[t];
        }
    }
    {
        // triples: indices, repeated spins, sizes, duplicates
        std::vector<std::array<int32_t, 3>> tk((size_t)d.t);
        for (int64_t k = 0; k < d.t; ++k) {
            std::array<int32_t, 3> v = {d.tri[3 * k], d.tri[3 * k + 1], d.tri[3 * k + 2]};
            for (int q = 0; q < 3; ++q)
                if (v[q] < 0 || v[q] >= n)
                    return fail(SG_EINVAL, "instance %d: triple %lld has a spin index out of range", idx,
                                (long long)k);
            if (v[0] == v[1] || v[0] == v[2] || v[1] == v[2])
                return fail(SG_EINVAL, "instance %d: triple %lld repeats a spin", idx, (long long)k);
            const int64_t c = std::llabs((int64_t)d.K[k]);
            if (c > kMaxCoef) w = true;
            total += c;
            std::sort(v.begin(), v.end());
            tk[k] = v;
        }
        std::sort(tk.begin(), tk.end());
        for (size_t k = 1; k < tk.size(); ++k)
            if (tk[k] == tk[k - 1])
                return fail(SG_EINVAL, "instance %d: triple (%d,%d,%d) given twice", idx, tk[k][0], tk[k][1],
                            tk[k][2]);
    }
    // every index is in range: the terms at each spin
    Incidence local;
    Incidence& I = inc ? *inc : local;
    build_incidence(d, I);  // this thread's scratch
    {
        // per spin: |h| + sum |coefficients| against the limits, and the
        // spin's edges to larger spins checked for a pair given twice
        std::vector<int64_t> dup_row(kHostThreads, -1), over_row(kHostThreads, -1), over_val(kHostThreads, 0);
        std::vector<int32_t> dup_col(kHostThreads, 0);
        std::vector<__int128> hpart(kHostThreads, 0);
        std::vector<char> big(kHostThreads, 0);
        parallel_ranges(n, [&](int64_t r0, int64_t r1) {
            const size_t slot = (size_t)(r0 * kHostThreads / std::max<int64_t>(n, 1));
            std::vector<int32_t> up;
            __int128 hs = 0;
            bool wf = false;
            for (int64_t i = r0; i < r1; ++i) {
                int64_t f = 0;
                up.clear();
                for (int64_t q = I.start[(size_t)i]; q < I.start[(size_t)i + 1]; ++q) {
                    f += std::llabs((int64_t)I.e[(size_t)q].c);
                    if (I.e[(size_t)q].b < 0 && I.e[(size_t)q].a > i) up.push_back(I.e[(size_t)q].a);
                }
                if (d.h) {
                    const int64_t c = std::llabs((int64_t)d.h[i]);
                    wf = wf || c > kMaxCoef;
                    f += c;
                    hs += c;
                }
                wf = wf || f > kMaxField;
                if (f > kMaxWideField && over_row[slot] < 0) {
                    over_row[slot] = i;
                    over_val[slot] = f;
                }
                if (up.size() > 1 && dup_row[slot] < 0) {
                    std::sort(up.begin(), up.end());
                    for (size_t k = 1; k < up.size(); ++k)
                        if (up[k] == up[k - 1]) {
                            dup_row[slot] = i;
                            dup_col[slot] = up[k];
                            break;
                        }
                }
            }
            hpart[slot] = hs;
            big[slot] = wf;
        });
        for (size_t t = 0; t < dup_row.size(); ++t)
            if (dup_row[t] >= 0)
                return fail(SG_EINVAL, "instance %d: edge (%lld,%d) given twice", idx, (long long)dup_row[t],
                            dup_col[t]);
        for (size_t t = 0; t < over_row.size(); ++t)
            if (over_row[t] >= 0)
                return fail(SG_ERANGE, "instance %d: spin %lld has |h|+sum|J|+sum|K| = %lld > %lld", idx,
                            (long long)over_row[t], (long long)over_val[t], (long long)kMaxWideField);
        for (size_t t = 0; t < hpart.size(); ++t) {
            total += hpart[t];
            w = w || big[t];
        }
    }
    if (total > (__int128)INT64_MAX)
        return fail(SG_ERANGE, "instance %d: sum|J| + sum|h| + sum|K| exceeds 2^63 - 1", idx);
    if (wide) *wide = w;
    return SG_OK;
}

sg_status check_lattice(const sg_instance_desc& d, int idx)
{
    const int dim = d.dims[2] ? 3 : 2;
    int64_t L[3] = {d.dims[0], d.dims[1], dim == 3 ? d.dims[2] : 1};
    for (int a = 0; a < dim; ++a)
        if (L[a] < 3) return fail(SG_EINVAL, "instance %d: lattice extent %lld < 3", idx, (long long)L[a]);
    if (L[0] * L[1] * L[2] != d.n)
        return fail(SG_EINVAL, "instance %d: lattice dims do not multiply to n", idx);
    if (d.m != (int64_t)dim * d.n)
        return fail(SG_EINVAL, "instance %d: a periodic %d-D lattice has %lld bonds, got %lld", idx, dim,
                    (long long)dim * d.n, (long long)d.m);
    // every edge joins two sites that differ by one step along one axis (in
    // 32-bit arithmetic: n < 2^31), checked over a few host threads
    const int32_t L1 = (int32_t)L[1], L2 = (int32_t)L[2], L12 = (int32_t)(L[1] * L[2]);
    const int32_t Lq[3] = {(int32_t)L[0], L1, L2};
    std::vector<int64_t> bad(kHostThreads, -1);
    parallel_ranges(d.m, [&](int64_t k0, int64_t k1) {
        const size_t slot = (size_t)(k0 * kHostThreads / std::max<int64_t>(d.m, 1));
        for (int64_t k = k0; k < k1; ++k) {
            const int32_t a = d.ei[k], b = d.ej[k];
            const int32_t ca[3] = {a / L12, (a / L2) % L1, a % L2};
            const int32_t cb[3] = {b / L12, (b / L2) % L1, b % L2};
            int diff = 0, ok = 1;
            for (int q = 0; q < 3; ++q) {
                if (ca[q] == cb[q]) continue;
                ++diff;
                const int32_t dd = (cb[q] - ca[q] + Lq[q]) % Lq[q];
                if (dd != 1 && dd != Lq[q] - 1) ok = 0;
            }
            if (diff != 1 || !ok) {
                bad[slot] = k;
                return;
            }
        }
    });
    for (int64_t k : bad)
        if (k >= 0)
            return fail(SG_EINVAL, "instance %d: edge %lld (%d,%d) is not a lattice bond", idx, (long long)k, d.ei[k],
                        d.ej[k]);
    return SG_OK;
}

// Lattice records for the implicit-neighbour schedules.  Accepted only when
// every extent is even, the colouring is the checkerboard and the
// colour-major relabel put site g at internal index colour(g)*n/2 + g/2 (true
// for the uniform-degree lattice); otherwise those schedules stay off.
void build_lattice(const sg_instance_desc& d, HostInst& q, const uint32_t* int_of)
{
    const int dim = d.dims[2] ? 3 : 2;
    int32_t L[3];
    if (dim == 3) {
        L[0] = d.dims[0]; L[1] = d.dims[1]; L[2] = d.dims[2];
    } else {
        L[0] = 1; L[1] = d.dims[0]; L[2] = d.dims[1];
    }
    for (int a = 3 - dim; a < 3; ++a)
        if (L[a] % 2) return;
    const int32_t n = d.n;
    const int32_t c0 = q.colour[0];
    if (c0 != 0 && c0 != 1) return;
    // site loops walk (x, y, z) incrementally from one division per range
    const int32_t stride[3] = {L[1] * L[2], L[2], 1};
    auto sites = [&](auto&& body) {
        parallel_ranges(n, [&](int64_t g0, int64_t g1) {
            int32_t c[3] = {(int32_t)g0 / stride[0], ((int32_t)g0 / L[2]) % L[1], (int32_t)g0 % L[2]};
            for (int64_t g = g0; g < g1; ++g) {
                if (!body((int32_t)g, c)) return;
                if (++c[2] == L[2]) {
                    c[2] = 0;
                    if (++c[1] == L[1]) {
                        c[1] = 0;
                        ++c[0];
                    }
                }
            }
        });
    };
    std::atomic<bool> ok{true};
    sites([&](int32_t g, const int32_t* c) {
        const int32_t col = (c[0] + c[1] + c[2] + c0) & 1;
        if (q.colour[g] != col || int_of[g] != (uint32_t)(col * (n / 2) + g / 2)) ok = false;
        return ok.load(std::memory_order_relaxed);
    });
    if (!ok) return;
    // each bond's J by its lower site and axis (every (site, axis) pair is one
    // bond, written once; the axis and direction follow from the index
    // difference, which is unique for extents >= 3), then every site's record
    // from its own and its lower neighbours' bonds
    std::vector<int8_t> bondJ((size_t)n * 3, 0);
    parallel_ranges(d.m, [&](int64_t k0, int64_t k1) {
        for (int64_t k = k0; k < k1; ++k) {
            const int32_t a = d.ei[k], b = d.ej[k];
            int32_t lo = -1, ax = 0;
            for (int x = 3 - dim; x < 3 && lo < 0; ++x) {
                const int32_t st = stride[x], wrap = (L[x] - 1) * stride[x];
                if (b - a == st || a - b == wrap) lo = a;        // b = a + e_x
                else if (a - b == st || b - a == wrap) lo = b;   // a = b + e_x
                ax = x;
            }
            bondJ[(size_t)lo * 3 + ax] = (int8_t)d.J[k];
        }
    });
    q.lat_rec.assign((size_t)n, 0);
    // with the records, whether the bit-plane form holds: every bond of the
    // lattice present with J = +-1, |h| <= 2
    std::atomic<bool> msc{true};
    sites([&](int32_t g, const int32_t* c) {
        uint64_t rc = 0;
        bool ok1 = true;
        for (int ax = 3 - dim; ax < 3; ++ax) {
            const int32_t down = c[ax] == 0 ? g + (L[ax] - 1) * stride[ax] : g - stride[ax];
            const int up_j = bondJ[(size_t)g * 3 + ax], down_j = bondJ[(size_t)down * 3 + ax];
            rc |= (uint64_t)(uint8_t)up_j << (8 * (2 * ax));
            rc |= (uint64_t)(uint8_t)down_j << (8 * (2 * ax + 1));
            ok1 = ok1 && (up_j == 1 || up_j == -1) && (down_j == 1 || down_j == -1);
        }
        const int hv = d.h ? (int)(int8_t)d.h[g] : 0;
        rc |= (uint64_t)(uint8_t)(int8_t)hv << 48;
        q.lat_rec[g] = rc;
        if (!ok1 || hv < -2 || hv > 2) msc.store(false, std::memory_order_relaxed);
        return true;
    });
    q.lat_msc = msc.load() ? 1 : 0;
    for (int a = 0; a < 3; ++a) q.lat_L[a] = L[a];
    q.lat_D = dim;
    q.lat_c0 = c0;
    q.lat_ok = 1;
    q.acc_slots = std::max(q.acc_slots, kMaxLatticeTiles);
}

sg_status ingest_dense(const sg_dense_desc& d, int idx, HostInst& q)
{
    if (d.n < 1 || d.n > 64) return fail(SG_EINVAL, "instance %d: n = %d (a dense instance has 1..64 spins)", idx, d.n);
    if (d.nterms < 0 || (d.nterms > 0 && (!d.mask || !d.coef)))
        return fail(SG_EINVAL, "instance %d: need mask and coef for %lld terms", idx, (long long)d.nterms);
    if (d.restarts < 1) return fail(SG_EINVAL, "instance %d: restarts must be >= 1", idx);
    if (d.restarts > kMaxRestarts) return fail(SG_ERANGE, "instance %d: restarts > %d", idx, kMaxRestarts);
    const int32_t n = d.n;
    const uint64_t all = n == 64 ? ~0ull : ((1ull << n) - 1);
    std::vector<uint64_t> sorted(d.mask, d.mask + d.nterms);
    std::sort(sorted.begin(), sorted.end());
    for (int64_t t = 0; t < d.nterms; ++t) {
        if (!d.mask[t]) return fail(SG_EINVAL, "instance %d: term %lld has no spin", idx, (long long)t);
        if (d.mask[t] & ~all)
            return fail(SG_EINVAL, "instance %d: term %lld names a spin >= n", idx, (long long)t);
        if (t > 0 && sorted[t] == sorted[t - 1])
            return fail(SG_EINVAL, "instance %d: a set of spins appears twice", idx);
    }
    // sum |coef| < 2^62 keeps energies and gains exact in int64
    unsigned long long acc = 0;
    for (int64_t t = 0; t < d.nterms; ++t) {
        const unsigned long long a = d.coef[t] < 0 ? 0ull - (unsigned long long)d.coef[t] : (unsigned long long)d.coef[t];
        if (a >= (1ull << 62) || acc + a >= (1ull << 62))
            return fail(SG_ERANGE, "instance %d: sum of |coef| reaches 2^62", idx);
        acc += a;
    }
    q.dense = 1;
    q.n = n;
    q.m = 0;
    q.t = 0;
    q.id = d.instance_id;
    q.R = d.restarts;
    q.t_mask.assign(d.mask, d.mask + d.nterms);
    q.t_coef.assign(d.coef, d.coef + d.nterms);
    // per-spin term lists: the other members and the coefficient
    q.d_start.assign((size_t)n + 1, 0);
    for (int64_t t = 0; t < d.nterms; ++t)
        for (int i = 0; i < n; ++i)
            if ((d.mask[t] >> i) & 1ull) q.d_start[i + 1]++;
    for (int i = 0; i < n; ++i) q.d_start[i + 1] += q.d_start[i];
    q.d_mask.assign((size_t)q.d_start[n], 0);
    q.d_coef.assign((size_t)q.d_start[n], 0);
    std::vector<int32_t> fill(q.d_start.begin(), q.d_start.end() - 1);
    for (int64_t t = 0; t < d.nterms; ++t)
        for (int i = 0; i < n; ++i)
            if ((d.mask[t] >> i) & 1ull) {
                q.d_mask[(size_t)fill[i]] = d.mask[t] & ~(1ull << i);
                q.d_coef[(size_t)fill[i]++] = d.coef[t];
            }
    // first-fit colouring over increasing index on the graph of shared terms
    uint64_t adj[64] = {0};
    for (int64_t t = 0; t < d.nterms; ++t)
        for (int i = 0; i < n; ++i)
            if ((d.mask[t] >> i) & 1ull) adj[i] |= d.mask[t] & ~(1ull << i);
    q.colour.assign((size_t)n, 0);
    int32_t C = 0;
    for (int i = 0; i < n; ++i) {
        uint64_t used = 0;
        for (int j = 0; j < i; ++j)
            if ((adj[i] >> j) & 1ull) used |= 1ull << q.colour[j];
        int c = 0;
        while ((used >> c) & 1ull) ++c;
        q.colour[i] = c;
        C = std::max(C, c + 1);
    }
    q.C = C;
    q.d_order.clear();
    for (int c = 0; c < C; ++c)
        for (int i = 0; i < n; ++i)
            if (q.colour[i] == c) q.d_order.push_back(i);
    q.ext_of.resize((size_t)n);
    for (int i = 0; i < n; ++i) q.ext_of[i] = (uint32_t)i;
    q.colour_slice.assign((size_t)C + 1, 0);
    q.h.assign((size_t)n, 0);
    return SG_OK;
}

sg_status ingest_wide(const sg_instance_desc& d, int idx, HostInst& q, const Incidence& P, const uint32_t* int_of,
                      const int64_t* es, const int64_t* ts);

sg_status ingest(const sg_instance_desc& d, int idx, HostInst& q)
{
    bool wide = false;
    Incidence P;
    sg_status st = validate(d, idx, &wide, &P);
    if (st != SG_OK) return st;
    q.n = d.n;
    q.m = d.m;
    q.t = d.t;
    q.id = d.instance_id;
    q.R = d.restarts;
    if (d.dims[0] || d.dims[1] || d.dims[2]) {
        st = check_lattice(d, idx);
        if (st != SG_OK) return st;
        q.lattice = 1;
        for (int a = 0; a < 3; ++a) q.dims[a] = d.dims[a];
    }
    const int32_t n = d.n;
    if (d.colour) {
        q.colour.assign(d.colour, d.colour + n);
        int32_t mx = -1;
        for (int32_t i = 0; i < n; ++i) {
            if (q.colour[i] < 0) return fail(SG_EINVAL, "instance %d: colour of spin %d is negative", idx, i);
            mx = std::max(mx, q.colour[i]);
        }
        for (int32_t i = 0; i < n; ++i)
            for (int64_t k = P.start[i]; k < P.start[i + 1]; ++k)
                for (const int32_t j : {P.e[k].a, P.e[k].b})
                    if (j >= 0 && q.colour[j] == q.colour[i])
                        return fail(SG_EINVAL,
                                    "instance %d: colouring is not proper (spins %d and %d share colour %d)", idx, i,
                                    j, q.colour[i]);
        q.C = mx + 1;
    } else if (q.lattice && d.t == 0 && d.dims[0] % 2 == 0 && d.dims[1] % 2 == 0 && d.dims[2] % 2 == 0) {
        // a periodic lattice with even extents (each >= 4) is bipartite, and
        // every site but the origin has a lower neighbour, so first-fit in
        // index order gives the checkerboard: colour (x + y + z) mod 2
        q.colour.resize((size_t)n);
        const int32_t L1 = d.dims[2] ? d.dims[1] : d.dims[0], L2 = d.dims[2] ? d.dims[2] : d.dims[1];
        parallel_ranges(n, [&](int64_t g0, int64_t g1) {
            int32_t z = (int32_t)(g0 % L2), y = (int32_t)((g0 / L2) % L1), x = (int32_t)(g0 / ((int64_t)L1 * L2));
            for (int64_t g = g0; g < g1; ++g) {
                q.colour[(size_t)g] = (x + y + z) & 1;
                if (++z == L2) {
                    z = 0;
                    if (++y == L1) {
                        y = 0;
                        ++x;
                    }
                }
            }
        });
        q.C = 2;
    } else {
        q.C = first_fit(P, n, q.colour);
    }

    // incidence counts (a spin's edges come before its triples)
    IngestScratch& S = ingest_scratch();
    int32_t* deg = S.deg.get((size_t)n);
    int32_t* tdeg = S.tdeg.get((size_t)n);
    parallel_ranges(n, [&](int64_t r0, int64_t r1) {
        for (int64_t i = r0; i < r1; ++i) {
            int32_t ne = 0;
            for (int64_t k = P.start[i]; k < P.start[i + 1] && P.e[k].b < 0; ++k) ++ne;
            deg[i] = ne;
            tdeg[i] = (int32_t)(P.start[i + 1] - P.start[i]) - ne;
        }
    });
    for (int32_t i = 0; i < n && !wide; ++i) wide = deg[i] > 65535 || tdeg[i] > 255;
    if (q.C > 65535) wide = true;
    q.wide = wide ? 1 : 0;
    // colour-major relabel, decreasing incidence inside a colour, stable
    q.ext_of.resize((size_t)n);
    std::iota(q.ext_of.begin(), q.ext_of.end(), 0u);
    {
        // order (colour ascending, couplings descending, triples descending,
        // index ascending) by three stable counting sorts, least significant
        // key first
        uint32_t* cur = q.ext_of.data();
        uint32_t* nxt = S.tmp.get((size_t)n);
        auto pass = [&](auto key, int64_t kmax, bool constant) {
            if (constant) return;  // one key value: the stable order stays
            std::vector<int64_t> cnt((size_t)kmax + 2, 0);
            for (int32_t k = 0; k < n; ++k) cnt[(size_t)key(cur[k]) + 1]++;
            for (int64_t v = 0; v <= kmax; ++v) cnt[(size_t)v + 1] += cnt[(size_t)v];
            for (int32_t k = 0; k < n; ++k) nxt[(size_t)cnt[(size_t)key(cur[k])]++] = cur[k];
            std::swap(cur, nxt);
        };
        int64_t dmax = 0, tmax = 0, dmin = INT64_MAX, tmin = INT64_MAX;
        for (int32_t i = 0; i < n; ++i) {
            dmax = std::max<int64_t>(dmax, deg[i]);
            tmax = std::max<int64_t>(tmax, tdeg[i]);
            dmin = std::min<int64_t>(dmin, deg[i]);
            tmin = std::min<int64_t>(tmin, tdeg[i]);
        }
        pass([&](uint32_t i) { return tmax - tdeg[i]; }, tmax, tmin == tmax);
        pass([&](uint32_t i) { return dmax - deg[i]; }, dmax, dmin == dmax);
        pass([&](uint32_t i) { return (int64_t)q.colour[i]; }, (int64_t)q.C - 1, q.C == 1);
        if (cur != q.ext_of.data()) std::memcpy(q.ext_of.data(), cur, (size_t)n * 4);
    }
    uint32_t* int_of = S.int_of.get((size_t)n);
    for (int32_t i = 0; i < n; ++i) int_of[q.ext_of[i]] = (uint32_t)i;

    // incidence lists in internal numbering
    int64_t* es = S.es.get((size_t)n + 1);
    int64_t* ts = S.ts.get((size_t)n + 1);
    es[0] = 0;
    ts[0] = 0;
    for (int32_t i = 0; i < n; ++i) {
        es[int_of[i] + 1] = deg[i];
        ts[int_of[i] + 1] = tdeg[i];
    }
    for (int32_t i = 0; i < n; ++i) {
        es[i + 1] += es[i];
        ts[i + 1] += ts[i];
    }
    if (q.wide) return ingest_wide(d, idx, q, P, int_of, es, ts);
    uint32_t* ew = S.ew.get(std::max<size_t>((size_t)es[n], 1));
    uint32_t* twa = S.twa.get(std::max<size_t>((size_t)ts[n], 1));
    uint32_t* twb = S.twb.get(std::max<size_t>((size_t)ts[n], 1));
    {
        // each thread writes the rows of its spins (external range) in
        // internal numbering, then sorts the internal rows of its range
        parallel_ranges(n, [&](int64_t r0, int64_t r1) {
            for (int64_t x = r0; x < r1; ++x) {
                const uint32_t ix = int_of[x];
                int64_t fe = es[ix], ft = ts[ix];
                for (int64_t k = P.start[x]; k < P.start[x + 1]; ++k) {
                    const uint32_t cb = (uint32_t)(uint8_t)(int8_t)P.e[k].c;
                    const uint32_t o1 = int_of[P.e[k].a];
                    if (P.e[k].b < 0) {
                        ew[fe++] = (o1 << 8) | cb;
                    } else {
                        const uint32_t o2 = int_of[P.e[k].b];
                        twa[ft] = (std::min(o1, o2) << 8) | cb;
                        twb[ft++] = std::max(o1, o2);
                    }
                }
            }
        });
        parallel_ranges(n, [&](int64_t r0, int64_t r1) {
            std::vector<std::pair<uint32_t, uint32_t>> tmp;
            for (int64_t i = r0; i < r1; ++i) {
                std::sort(ew + es[i], ew + es[i + 1]);
                // order triple entries of a row by partner (pairs sorted together)
                if (ts[i + 1] - ts[i] < 2) continue;
                tmp.clear();
                for (int64_t k = ts[i]; k < ts[i + 1]; ++k) tmp.emplace_back(twa[k], twb[k]);
                std::sort(tmp.begin(), tmp.end());
                for (int64_t k = ts[i]; k < ts[i + 1]; ++k) {
                    twa[k] = tmp[k - ts[i]].first;
                    twb[k] = tmp[k - ts[i]].second;
                }
            }
        });
    }
    // fields
    q.h.assign((size_t)n, 0);
    if (d.h)
        for (int32_t i = 0; i < n; ++i) q.h[int_of[i]] = (int8_t)d.h[i];

    // sliced layout, colour by colour
    std::vector<int32_t> cstart((size_t)q.C + 1, 0);
    for (int32_t i = 0; i < n; ++i) cstart[q.colour[i] + 1]++;
    for (int32_t c = 0; c < q.C; ++c) cstart[c + 1] += cstart[c];
    q.colour_slice.assign((size_t)q.C + 1, 0);
    uint64_t ebase = 0, tbase = 0;
    int32_t maxblocks = 1;
    for (int32_t c = 0; c < q.C; ++c) {
        q.colour_slice[c] = (int32_t)q.slices.size();
        for (int32_t r0 = cstart[c]; r0 < cstart[c + 1]; r0 += sg::kSlice) {
            const int32_t rows = std::min(sg::kSlice, cstart[c + 1] - r0);
            int32_t w = 0, tw = 0;
            for (int32_t l = 0; l < rows; ++l) {
                w = std::max<int32_t>(w, (int32_t)(es[r0 + l + 1] - es[r0 + l]));
                tw = std::max<int32_t>(tw, (int32_t)(ts[r0 + l + 1] - ts[r0 + l]));
            }
            sg::Slice S;
            S.row0 = (uint32_t)r0;
            S.ebase = (uint32_t)ebase;
            S.tbase = (uint32_t)tbase;
            S.ew = (uint16_t)w;
            S.tw = (uint8_t)tw;
            S.rows = (uint8_t)rows;
            q.slices.push_back(S);
            ebase += (uint64_t)w * sg::kSlice;
            tbase += (uint64_t)tw * sg::kSlice;
            if (ebase > 0xFFFFFFFFull || tbase > 0xFFFFFFFFull)
                return fail(SG_ERANGE, "instance %d: coupling layout exceeds 2^32 words", idx);
        }
        const int32_t ns = (int32_t)q.slices.size() - q.colour_slice[c];
        maxblocks = std::max(maxblocks, (ns + sg::kPhaseWaves - 1) / sg::kPhaseWaves);
    }
    q.colour_slice[q.C] = (int32_t)q.slices.size();
    q.nslots = maxblocks;
    q.acc_slots = maxblocks;
    q.nbr.assign((size_t)std::max<uint64_t>(ebase, 1), 0u);
    q.ta.assign((size_t)std::max<uint64_t>(tbase, 1), 0u);
    q.tb.assign((size_t)std::max<uint64_t>(tbase, 1), 0u);
    // term list of small instances, for the energy of one replica per lane
    q.eterm.clear();
    q.n_eh = q.n_ee = q.n_et = 0;
    q.max_w = 0;
    for (int32_t i = 0; i < n; ++i) {
        int64_t W = std::abs((int32_t)q.h[i]);
        for (int64_t k = es[i]; k < es[i + 1]; ++k) W += std::abs((int32_t)(int8_t)(ew[k] & 0xFFu));
        for (int64_t k = ts[i]; k < ts[i + 1]; ++k) W += std::abs((int32_t)(int8_t)(twa[k] & 0xFFu));
        q.max_w = std::max(q.max_w, W);
    }
    q.bits_ok = 0;
    if (n <= kLaneStartMaxN) {
        bool ok = true;
        for (int32_t i = 0; i < n && ok; ++i) {
            int32_t W = std::abs((int32_t)q.h[i]);
            ok = W <= 15;
            for (int64_t k = es[i]; k < es[i + 1] && ok; ++k) {
                const int32_t c = std::abs((int32_t)(int8_t)(ew[k] & 0xFFu));
                ok = c <= 15;
                W += c;
            }
            for (int64_t k = ts[i]; k < ts[i + 1] && ok; ++k) {
                const int32_t c = std::abs((int32_t)(int8_t)(twa[k] & 0xFFu));
                ok = c <= 15;
                W += c;
            }
            ok = ok && W <= 255;
        }
        q.bits_ok = ok ? 1 : 0;
    }
    if (n <= kLaneStartMaxN) {
        for (int32_t i = 0; i < n; ++i)
            if (q.h[i]) q.eterm.push_back((uint32_t)i | ((uint32_t)(uint8_t)q.h[i] << 22));
        q.n_eh = (int32_t)q.eterm.size();
        for (int32_t i = 0; i < n; ++i)
            for (int64_t k = es[i]; k < es[i + 1]; ++k) {
                const uint32_t j = ew[k] >> 8, Jb = ew[k] & 0xFFu;
                if ((int32_t)j > i && Jb) q.eterm.push_back((uint32_t)i | (j << 11) | (Jb << 22));
            }
        q.n_ee = (int32_t)q.eterm.size() - q.n_eh;
        for (int32_t i = 0; i < n; ++i)
            for (int64_t k = ts[i]; k < ts[i + 1]; ++k) {
                const uint32_t a = twa[k] >> 8, Kb = twa[k] & 0xFFu, b = twb[k];
                if ((int32_t)a > i && (int32_t)b > i && Kb) {
                    q.eterm.push_back((uint32_t)i | (a << 11) | (Kb << 22));
                    q.eterm.push_back(b);
                    ++q.n_et;
                }
            }
    }
    parallel_ranges((int64_t)q.slices.size(), [&](int64_t s0, int64_t s1) {
        for (int64_t si = s0; si < s1; ++si) {
            const sg::Slice& S = q.slices[(size_t)si];
            for (int32_t l = 0; l < S.rows; ++l) {
                const int32_t i = (int32_t)S.row0 + l;
                for (int64_t k = es[i]; k < es[i + 1]; ++k) q.nbr[S.ebase + (k - es[i]) * sg::kSlice + l] = ew[k];
                for (int64_t k = ts[i]; k < ts[i + 1]; ++k) {
                    q.ta[S.tbase + (k - ts[i]) * sg::kSlice + l] = twa[k];
                    q.tb[S.tbase + (k - ts[i]) * sg::kSlice + l] = twb[k];
                }
            }
        }
    });
    if (q.lattice && q.t == 0) build_lattice(d, q, int_of);
    return SG_OK;
}

// The wide form: the rows of the packed form with the partner index and the
// coefficient in separate 32-bit words (int_of, es, ts: the relabel and the
// per-row incidence offsets in internal numbering).
sg_status ingest_wide(const sg_instance_desc& d, int idx, HostInst& q, const Incidence& P, const uint32_t* int_of,
                      const int64_t* es, const int64_t* ts)
{
    const int32_t n = d.n;
    std::vector<uint32_t> wp((size_t)es[n]), wa((size_t)ts[n]), wb((size_t)ts[n]);
    std::vector<int32_t> wj((size_t)es[n]), wk((size_t)ts[n]);
    // each spin's terms in input order, in internal numbering
    parallel_ranges(n, [&](int64_t r0, int64_t r1) {
        for (int64_t x = r0; x < r1; ++x) {
            const uint32_t ix = int_of[x];
            int64_t fe = es[ix], ft = ts[ix];
            for (int64_t k = P.start[x]; k < P.start[x + 1]; ++k) {
                const uint32_t o1 = int_of[P.e[k].a];
                if (P.e[k].b < 0) {
                    wp[fe] = o1;
                    wj[fe++] = P.e[k].c;
                } else {
                    const uint32_t o2 = int_of[P.e[k].b];
                    wa[ft] = std::min(o1, o2);
                    wb[ft] = std::max(o1, o2);
                    wk[ft++] = P.e[k].c;
                }
            }
        }
    });
    q.w_h.assign((size_t)n, 0);
    if (d.h)
        for (int32_t i = 0; i < n; ++i) q.w_h[int_of[i]] = d.h[i];
    std::vector<int64_t> cstart((size_t)q.C + 1, 0);
    for (int32_t i = 0; i < n; ++i) cstart[q.colour[i] + 1]++;
    for (int32_t c = 0; c < q.C; ++c) cstart[c + 1] += cstart[c];
    q.colour_slice.assign((size_t)q.C + 1, 0);
    q.w_slices.clear();
    uint64_t ebase = 0, tbase = 0;
    int64_t maxblocks = 1;
    for (int32_t c = 0; c < q.C; ++c) {
        if (q.w_slices.size() > (size_t)INT32_MAX - 1)
            return fail(SG_ERANGE, "instance %d: more than 2^31 - 1 row slices", idx);
        q.colour_slice[c] = (int32_t)q.w_slices.size();
        for (int64_t r0 = cstart[c]; r0 < cstart[c + 1]; r0 += sg::kSlice) {
            const int32_t rows = (int32_t)std::min<int64_t>(sg::kSlice, cstart[c + 1] - r0);
            int64_t w = 0, tw = 0;
            for (int32_t l = 0; l < rows; ++l) {
                w = std::max<int64_t>(w, es[r0 + l + 1] - es[r0 + l]);
                tw = std::max<int64_t>(tw, ts[r0 + l + 1] - ts[r0 + l]);
            }
            sg::WSlice S;
            S.ebase = ebase;
            S.tbase = tbase;
            S.row0 = (uint32_t)r0;
            S.ew = (uint32_t)w;
            S.tw = (uint32_t)tw;
            S.rows = (uint32_t)rows;
            q.w_slices.push_back(S);
            ebase += (uint64_t)w * sg::kSlice;
            tbase += (uint64_t)tw * sg::kSlice;
        }
        const int64_t ns = (int64_t)q.w_slices.size() - q.colour_slice[c];
        maxblocks = std::max<int64_t>(maxblocks, (ns + sg::kPhaseWaves - 1) / sg::kPhaseWaves);
    }
    if (q.w_slices.size() > (size_t)INT32_MAX) return fail(SG_ERANGE, "instance %d: more than 2^31 - 1 row slices", idx);
    q.colour_slice[q.C] = (int32_t)q.w_slices.size();
    q.nslots = (int32_t)maxblocks;
    q.acc_slots = (int32_t)maxblocks;
    q.w_nbr.assign((size_t)std::max<uint64_t>(ebase, 1), 0u);
    q.w_J.assign((size_t)std::max<uint64_t>(ebase, 1), 0);
    q.w_ta.assign((size_t)std::max<uint64_t>(tbase, 1), 0u);
    q.w_tb.assign((size_t)std::max<uint64_t>(tbase, 1), 0u);
    q.w_K.assign((size_t)std::max<uint64_t>(tbase, 1), 0);
    q.max_w = 0;
    for (const sg::WSlice& S : q.w_slices) {
        for (uint32_t l = 0; l < S.rows; ++l) {
            const int64_t i = (int64_t)S.row0 + l;
            int64_t W = std::llabs((int64_t)q.w_h[(size_t)i]);
            for (int64_t k = es[i]; k < es[i + 1]; ++k) {
                const uint64_t at = S.ebase + (uint64_t)(k - es[i]) * sg::kSlice + l;
                q.w_nbr[at] = wp[k];
                q.w_J[at] = wj[k];
                W += std::llabs((int64_t)wj[k]);
            }
            for (int64_t k = ts[i]; k < ts[i + 1]; ++k) {
                const uint64_t at = S.tbase + (uint64_t)(k - ts[i]) * sg::kSlice + l;
                q.w_ta[at] = wa[k];
                q.w_tb[at] = wb[k];
                q.w_K[at] = wk[k];
                W += std::llabs((int64_t)wk[k]);
            }
            q.max_w = std::max(q.max_w, W);
        }
    }
    // the packed arrays stay empty placeholders
    q.slices.clear();
    q.nbr.assign(1, 0u);
    q.ta.assign(1, 0u);
    q.tb.assign(1, 0u);
    q.h.assign(1, 0);
    q.eterm.clear();
    q.n_eh = q.n_ee = q.n_et = 0;
    q.bits_ok = 0;
    q.lat_ok = 0;
    return SG_OK;
}

// Replicas of this instance may start (and recompute energies) one lane per replica.
bool lane_start_candidate(const HostInst& q)
{
    return !q.dense && !q.wide && q.n <= kLaneStartMaxN && q.R >= kLaneStartMinR;
}

// The pass kernel with one replica per lane takes instances of at most 1024
// spins (tags of the move order fit a byte) whose every half-gain -s_i f_i
// fits a byte, with at most 16 couplings and 6 hyper-couplings on a spin
// (its rows of fixed width).
void fml_counts(const HostInst& q, int32_t& dmax, int32_t& tmax)
{
    dmax = tmax = 0;
    for (const sg::Slice& S : q.slices)
        for (uint32_t l = 0; l < S.rows; ++l) {
            int32_t c = 0, t = 0;
            for (uint32_t k = 0; k < S.ew; ++k) c += (q.nbr[S.ebase + (size_t)k * sg::kSlice + l] & 0xFFu) != 0;
            for (uint32_t k = 0; k < S.tw; ++k) t += (q.ta[S.tbase + (size_t)k * sg::kSlice + l] & 0xFFu) != 0;
            dmax = std::max(dmax, c);
            tmax = std::max(tmax, t);
        }
}

// Instances the large-instance pass kernel takes: beyond one wavefront's LDS
// (more than kFmMaxN spins) and within its 2^24 - 1 (upper-level keys in
// LDS).  dc, tt: the widest row's nonzero couplings and hyper-couplings.
constexpr int32_t kFmBigMaxN = (1 << 24) - 1;

bool fmb_candidate(const HostInst& q, int32_t* dc = nullptr, int32_t* tt = nullptr)
{
    if (q.dense || q.n <= kFmMaxN || q.n > kFmBigMaxN) return false;
    int32_t d = 0, t = 0;
    if (!q.wide) {
        for (const sg::Slice& S : q.slices)
            for (int32_t l = 0; l < S.rows; ++l) {
                int32_t cd = 0, ct = 0;
                for (int32_t k = 0; k < S.ew; ++k) cd += (q.nbr[S.ebase + (size_t)k * sg::kSlice + l] & 0xFFu) != 0;
                for (int32_t k = 0; k < S.tw; ++k) ct += (q.ta[S.tbase + (size_t)k * sg::kSlice + l] & 0xFFu) != 0;
                d = std::max(d, cd);
                t = std::max(t, ct);
            }
    } else {
        for (const sg::WSlice& S : q.w_slices)
            for (uint32_t l = 0; l < S.rows; ++l) {
                int32_t cd = 0, ct = 0;
                for (uint32_t k = 0; k < S.ew; ++k) cd += q.w_J[S.ebase + (size_t)k * sg::kSlice + l] != 0;
                for (uint32_t k = 0; k < S.tw; ++k) ct += q.w_K[S.tbase + (size_t)k * sg::kSlice + l] != 0;
                d = std::max(d, cd);
                t = std::max(t, ct);
            }
    }
    if (dc) *dc = d;
    if (tt) *tt = t;
    return true;
}

int32_t fmb_stride(const HostInst& q) { return q.wide ? 1 + 2 * q.fmb_dc + 3 * q.fmb_tt : 1 + q.fmb_dc + 2 * q.fmb_tt; }

// The large-instance pass kernel's rows (FmbRows): per spin in external order
// its field, its nonzero couplings and hyper-couplings with partners in
// external order, zero-padded to q.fmb_dc and q.fmb_tt.
void build_fmb_rows(const HostInst& q, std::vector<uint32_t>& out)
{
    const int32_t dc = q.fmb_dc, stride = fmb_stride(q);
    out.assign((size_t)q.n * stride, 0u);
    if (!q.wide) {
        for (const sg::Slice& S : q.slices)
            for (int32_t l = 0; l < S.rows; ++l) {
                const int32_t i = (int32_t)S.row0 + l;
                uint32_t* row = out.data() + (size_t)q.ext_of[(size_t)i] * stride;
                row[0] = (uint32_t)(uint8_t)q.h[(size_t)i];
                int32_t c = 0, t = 0;
                for (int32_t k = 0; k < S.ew; ++k) {
                    const uint32_t w = q.nbr[S.ebase + (size_t)k * sg::kSlice + l];
                    if (w & 0xFFu) row[1 + c++] = (q.ext_of[w >> 8] << 8) | (w & 0xFFu);
                }
                for (int32_t k = 0; k < S.tw; ++k) {
                    const uint32_t wa = q.ta[S.tbase + (size_t)k * sg::kSlice + l];
                    if (!(wa & 0xFFu)) continue;
                    const uint32_t b = q.tb[S.tbase + (size_t)k * sg::kSlice + l];
                    row[1 + dc + 2 * t] = (q.ext_of[wa >> 8] << 8) | (wa & 0xFFu);
                    row[2 + dc + 2 * t] = q.ext_of[b];
                    ++t;
                }
            }
        return;
    }
    for (const sg::WSlice& S : q.w_slices)
        for (uint32_t l = 0; l < S.rows; ++l) {
            const uint32_t i = S.row0 + l;
            uint32_t* row = out.data() + (size_t)q.ext_of[i] * stride;
            row[0] = (uint32_t)q.w_h[i];
            int32_t c = 0, t = 0;
            for (uint32_t k = 0; k < S.ew; ++k) {
                const uint64_t at = S.ebase + (uint64_t)k * sg::kSlice + l;
                if (!q.w_J[at]) continue;
                row[1 + 2 * c] = q.ext_of[q.w_nbr[at]];
                row[2 + 2 * c] = (uint32_t)q.w_J[at];
                ++c;
            }
            for (uint32_t k = 0; k < S.tw; ++k) {
                const uint64_t at = S.tbase + (uint64_t)k * sg::kSlice + l;
                if (!q.w_K[at]) continue;
                uint32_t* t3 = row + 1 + 2 * dc + 3 * t;
                t3[0] = q.ext_of[q.w_ta[at]];
                t3[1] = q.ext_of[q.w_tb[at]];
                t3[2] = (uint32_t)q.w_K[at];
                ++t;
            }
        }
}

bool fml_candidate(const HostInst& q)
{
    if (q.dense || q.wide || q.n > kFmlMaxN || q.max_w > kFmlMaxW) return false;
    int32_t d, t;
    fml_counts(q, d, t);
    return d <= 16 && t <= 6;
}

// byte offset of spin j in the lane-interleaved gain words of the lane kernel
inline uint32_t fml_fb(uint32_t j) { return (j >> 2) << 8 | (j & 3u); }

// Appends the term rows of one instance in external order: per spin e a word
// h_e & 255 | couplings << 8 | hyper-couplings << 16 (padded to an even
// count), then per spin dc coupling words fb(j) << 16 | (j & 31) << 11 |
// J & 255, then per spin tt pairs of words, one hyper-coupling each:
// (fb(a) << 16 | fb(b), (a & 31) << 24 | (b & 31) << 16 | K & 255); partners
// as external indices.  Unused entries name spin e itself with coefficient 0
// (the sliced layout's zero padding is left out).  dc (4, 6, 8 or 16) and tt
// (0, 2, 4 or 6) are widths the lane kernel is built for, shared by every
// instance of the handle so that one launch runs them all.
void build_fml(const HostInst& q, std::vector<uint32_t>& out, int32_t dc, int32_t tt)
{
    const int32_t n = q.n;
    const size_t hn = ((size_t)n + 1) & ~(size_t)1;
    const size_t base = out.size();
    out.resize(base + hn + (size_t)n * (size_t)(dc + 2 * tt), 0u);
    uint32_t* w = out.data() + base;
    uint32_t* cw = w + hn;
    uint32_t* tw = cw + (size_t)n * (size_t)dc;
    for (const sg::Slice& S : q.slices)
        for (uint32_t l = 0; l < S.rows; ++l) {
            const uint32_t i = S.row0 + l, e = q.ext_of[i];
            const uint32_t self_c = fml_fb(e) << 16 | (e & 31u) << 11;
            uint32_t* cr = cw + (size_t)e * (size_t)dc;
            uint32_t* ce = cr + dc;
            uint32_t nc = 0, nt = 0;
            for (uint32_t k = 0; k < S.ew; ++k) {
                const uint32_t x = q.nbr[S.ebase + (size_t)k * sg::kSlice + l];
                if (!(x & 0xFFu)) continue;
                const uint32_t j = q.ext_of[x >> 8];
                *cr++ = fml_fb(j) << 16 | (j & 31u) << 11 | (x & 0xFFu);
                ++nc;
            }
            while (cr < ce) *cr++ = self_c;
            uint32_t* tr = tw + (size_t)e * 2 * (size_t)tt;
            uint32_t* te = tr + 2 * (size_t)tt;
            for (uint32_t k = 0; k < S.tw; ++k) {
                const size_t at = S.tbase + (size_t)k * sg::kSlice + l;
                const uint32_t x = q.ta[at];
                if (!(x & 0xFFu)) continue;
                const uint32_t a = q.ext_of[x >> 8], b = q.ext_of[q.tb[at]];
                *tr++ = fml_fb(a) << 16 | fml_fb(b);
                *tr++ = (a & 31u) << 24 | (b & 31u) << 16 | (x & 0xFFu);
                ++nt;
            }
            while (tr < te) {
                *tr++ = fml_fb(e) << 16 | fml_fb(e);
                *tr++ = (e & 31u) << 24 | (e & 31u) << 16;
            }
            w[e] = ((uint32_t)(int32_t)q.h[i] & 0xFFu) | nc << 8 | nt << 16;
        }
}

void layout(sg_ctx* H)
{
    // the lane path keeps one wavefront per 64 replicas busy with a whole
    // instance: it pays off only with enough such wavefronts to fill the GPU
    int64_t lane_reps = 0;
    for (const HostInst& q : H->insts)
        if (lane_start_candidate(q)) lane_reps += q.R;
    H->lanes_on = lane_reps >= kLaneStartMinTotal;
    auto lane_start = [&](const HostInst& q) { return H->lanes_on && lane_start_candidate(q); };
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        const uint64_t o = off;
        off = align_up(off + std::max<uint64_t>(bytes, 1));
        return o;
    };
    int64_t max_slots = 1;
    for (HostInst& q : H->insts) {
        if (q.wide) {
            q.off_wnbr = take(q.w_nbr.size() * 4);
            q.off_wJ = take(q.w_J.size() * 4);
            q.off_wta = take(q.w_ta.size() * 4);
            q.off_wtb = take(q.w_tb.size() * 4);
            q.off_wK = take(q.w_K.size() * 4);
            q.off_wh = take(q.w_h.size() * 4);
            q.off_wslices = take(q.w_slices.size() * sizeof(sg::WSlice));
        }
        q.off_nbr = take(q.nbr.size() * 4);
        q.off_ta = take(q.ta.size() * 4);
        q.off_tb = take(q.tb.size() * 4);
        q.off_h = take(q.h.size());
        q.off_ext = take((uint64_t)q.n * 4);
        q.off_slices = take(q.slices.size() * sizeof(sg::Slice));
        q.off_eterm = take(q.eterm.size() * 4);
        q.spin_stride = align_up((uint64_t)q.n);
        q.off_spins = take(q.spin_stride * (uint64_t)q.R);
        q.off_acc = take((uint64_t)q.R * q.acc_slots * 16);
        q.field_stride = H->fields_ws ? align_up((uint64_t)q.n * 4) / 4 : 0;
        q.off_fields = H->fields_ws ? take(q.field_stride * 4 * (uint64_t)q.R) : 0;
        if (q.dense) {
            q.off_dstart = take(q.d_start.size() * 4);
            q.off_dmask = take(q.d_mask.size() * 8);
            q.off_dcoef = take(q.d_coef.size() * 8);
            q.off_tmask = take(q.t_mask.size() * 8);
            q.off_tcoef = take(q.t_coef.size() * 8);
            q.off_dorder = take(q.d_order.size() * 4);
        }
        if (q.lat_ok) {
            q.off_lat_rec = take((uint64_t)q.n * 8);
            // two copies of one 8-byte word (epoch tag and bits) per interior z-row of
            // every tile (z extent >= 4 sites)
            q.lat_g_bytes = ((uint64_t)q.n / 4 + 4096) * 8 * 2 * q.R;
            q.off_lat_g = take(q.lat_g_bytes);
            q.off_lat_cnt = take((uint64_t)q.R * kConvChunk * 8);

        }
        max_slots = std::max<int64_t>(max_slots, (int64_t)q.R * q.nslots);
    }
    H->off_reps = take((uint64_t)H->total_reps * sizeof(sg::RepState));
    H->off_stats = take(sizeof(sg::CallStats));
    H->off_flag = take(64);
    H->off_err = take(64);
    H->off_eout = take((uint64_t)H->total_reps * 8);
    H->off_slots = take((uint64_t)max_slots * 8);
    const uint64_t ni = H->insts.size();
    H->n_block_item_cap = 0;
    H->ctab_len = 0;
    for (const HostInst& q : H->insts) {
        H->n_block_item_cap += (q.R + 63) / 64;
        H->ctab_len += q.C + 1;
    }
    H->h_fml.clear();
    H->fm_item_cap = 0;
    int32_t fdmax = 0, ftmax = 0;
    for (HostInst& q : H->insts) {
        q.fml_off = UINT64_MAX;
        if (!H->fml_ws || !fml_candidate(q)) continue;
        q.fml_off = 0;
        int32_t d, t;
        fml_counts(q, d, t);
        fdmax = std::max(fdmax, d);
        ftmax = std::max(ftmax, t);
    }
    const int32_t fdc = fdmax <= 4 ? 4 : fdmax <= 6 ? 6 : fdmax <= 8 ? 8 : 16;
    const int32_t ftt = ftmax == 0 ? 0 : ftmax <= 2 ? 2 : ftmax <= 4 ? 4 : 6;
    for (HostInst& q : H->insts) {
        if (q.fml_off == UINT64_MAX) continue;
        q.fml_off = H->h_fml.size();
        q.fml_dc = fdc;
        q.fml_tt = ftt;
        build_fml(q, H->h_fml, fdc, ftt);
        H->fm_item_cap += (q.R + 63) / 64;
    }
    H->off_fml = take(H->h_fml.size() * 4);
    H->off_fmitems = take((uint64_t)H->fm_item_cap * sizeof(sg::BlockItem));
    H->off_tab = take(ni * sizeof(sg::InstTab));
    H->off_ctab = take((uint64_t)H->ctab_len * 4);
    H->off_bitems = take((uint64_t)H->n_block_item_cap * sizeof(sg::BlockItem));
    H->off_qitems = take((uint64_t)H->total_reps * sizeof(sg::QueueItem));
    H->off_qcnt = take(64);
    H->off_rep_inst = take((uint64_t)H->total_reps * 4);
    H->off_tbase = take((uint64_t)H->insts.size() * 4);
    H->h_sunits.clear();
    H->h_eunits.clear();
    H->h_esegs.clear();
    for (size_t k = 0; k < H->insts.size(); ++k) {
        const HostInst& q = H->insts[k];
        if (q.dense || lane_start(q)) continue;
        for (int32_t r = 0; r < q.R; ++r) {
            const int64_t g = q.rep_base + r;
            for (int32_t i0 = 0; i0 < q.n; i0 += 1024) H->h_sunits.push_back(sg::StartUnit{g, (int32_t)k, i0});
            if (q.wide) continue;  // energies of the wide form: the wide energy pass
            const int64_t u0 = (int64_t)H->h_eunits.size();
            for (int32_t s0 = 0; s0 < (int32_t)q.slices.size(); s0 += 4)
                H->h_eunits.push_back(sg::StartUnit{g, (int32_t)k, s0});
            H->h_esegs.push_back(sg::EnergySeg{g, u0, (int32_t)((int64_t)H->h_eunits.size() - u0), 0});
        }
    }
    H->off_sunits = take(H->h_sunits.size() * sizeof(sg::StartUnit));
    H->off_eunits = take(H->h_eunits.size() * sizeof(sg::StartUnit));
    H->off_esegs = take(H->h_esegs.size() * sizeof(sg::EnergySeg));
    H->off_eparts = take(H->h_eunits.size() * 8);
    H->h_litems.clear();
    H->lane_nmax = 1;
    for (size_t k = 0; k < H->insts.size(); ++k) {
        const HostInst& q = H->insts[k];
        if (!lane_start(q)) continue;
        H->lane_nmax = std::max(H->lane_nmax, q.n);
        for (int32_t r0 = 0; r0 < q.R; r0 += 64)
            H->h_litems.push_back(sg::BlockItem{(int32_t)k, r0, std::min(64, q.R - r0), 0});
    }
    H->off_litems = take(H->h_litems.size() * sizeof(sg::BlockItem));
    H->h_ditems.clear();
    H->dense_nmax = 1;
    for (size_t k = 0; k < H->insts.size(); ++k) {
        const HostInst& q = H->insts[k];
        if (!q.dense) continue;
        H->dense_nmax = std::max(H->dense_nmax, q.n);
        for (int32_t r0 = 0; r0 < q.R; r0 += 64)
            H->h_ditems.push_back(sg::BlockItem{(int32_t)k, r0, std::min(64, q.R - r0), 0});
    }
    H->off_dtab = take(ni * sizeof(sg::DenseTab));
    H->off_ditems = take(H->h_ditems.size() * sizeof(sg::BlockItem));
    H->off_best_E = take(ni * 8);
    H->off_best_r = take(ni * 4);
    H->off_solve = take(64 + ni * 12);  // sg_solve's results: call totals, best energies, best restarts
    H->off_rep_base = take(ni * 8);
    H->off_restarts = take(ni * 4);
    // the large-instance pass kernel (fm_slots replicas at once): per slot
    // the half-gains, the move list and the leaf keys of the largest such
    // instance; per instance its external -> internal map
    H->fmb_nmax = 0;
    H->fmb_reps = 0;
    for (HostInst& q : H->insts) {
        q.off_fmb_rows = UINT64_MAX;
        if (H->fm_slots <= 0 || !fmb_candidate(q, &q.fmb_dc, &q.fmb_tt)) continue;
        H->fmb_nmax = std::max(H->fmb_nmax, q.n);
        H->fmb_reps += q.R;
        q.off_fmb_rows = take((uint64_t)q.n * fmb_stride(q) * 4);
    }
    if (H->fmb_nmax > 0) {
        const int64_t slots = std::min<int64_t>(H->fm_slots, H->fmb_reps);
        H->fmb_slot_spins = (H->fmb_nmax + 255) / 256 * 256;
        H->fmb_slot_leaves = (H->fmb_nmax + 63) / 64;
        H->off_fmb_half = take((uint64_t)slots * H->fmb_slot_spins * 4);
        H->off_fmb_moves = take((uint64_t)slots * H->fmb_slot_spins * 4);
        H->off_fmb_spin = take((uint64_t)slots * H->fmb_slot_spins);
        H->off_fmb_leaf = take((uint64_t)slots * H->fmb_slot_leaves * 8);
        H->off_fmb_ptr = take(ni * sizeof(sg::FmbRows));
        H->off_fmb_items = take((uint64_t)H->fmb_reps * sizeof(sg::QueueItem));
        H->off_fmb_cnt = take(64);
    }
    H->bytes = off;
}

sg_status need_bound(sg_handle H)
{
    if (!H) return fail(SG_EINVAL, "null handle");
    if (!H->bound) return fail(SG_ESTATE, "handle is not bound to device memory (call sg_bind)");
    return SG_OK;
}

sg_status check_inst(sg_handle H, int32_t inst, int32_t r)
{
    if (inst < 0 || inst >= (int32_t)H->insts.size())
        return fail(SG_EINVAL, "instance index %d out of range [0,%zu)", inst, H->insts.size());
    if (r < 0 || r >= H->insts[inst].R)
        return fail(SG_EINVAL, "restart %d out of range [0,%d)", r, H->insts[inst].R);
    return SG_OK;
}

// ---------------------------------------------------------------------------
// run driver: one kernel launch per colour phase, instance by instance

sg_status run_phase_schedule(sg_handle H, const sg_run_params* p, const std::vector<int>& which, bool inc = false)
{
    hipStream_t st = H->stream;
    sg::CallStats* cs = H->at<sg::CallStats>(H->off_stats);
    uint32_t* flag = H->at<uint32_t>(H->off_flag);
    for (int qi : which) {
        const HostInst& q = H->insts[qi];
        const sg::InstDev I = H->view(q);
        sg::RepState* rs = H->reps() + q.rep_base;
        int8_t* spins = H->at<int8_t>(q.off_spins);
        int64_t* acc = H->at<int64_t>(q.off_acc);
        SG_HIP(sg::launch_begin(rs, q.R, acc, (int64_t)q.R * q.acc_slots * 2, st), "begin kernel");
        if (qi == which.front()) {
            SG_HIP(hipEventRecord(H->evh0, st), "event record");
            H->hot_launches = 0;
        }
        int32_t* F = inc ? H->at<int32_t>(q.off_fields) : nullptr;
        const int64_t fstride = (int64_t)q.field_stride;
        if (inc) SG_HIP(sg::launch_fields(I, spins, (int64_t)q.spin_stride, q.R, F, fstride, st), "field kernel");
        int T = 0;
        const sg::WideDev W = q.wide ? H->wview(q) : sg::WideDev{};
        auto sweeps = [&](int from, int to) -> sg_status {
            for (int t = from; t < to; ++t)
                for (int32_t c = 0; c < q.C; ++c) {
                    const int s0 = q.colour_slice[c], ns = q.colour_slice[c + 1] - s0;
                    if (q.wide)
                        SG_HIP(sg::launch_wide_phase(W, spins, (int64_t)q.spin_stride, rs, q.R, acc, q.acc_slots, s0,
                                                     ns, t, p->seed, p->rule, p->until_converged, st),
                               "wide phase kernel");
                    else
                        SG_HIP(sg::launch_phase(I, spins, (int64_t)q.spin_stride, rs, q.R, acc, q.acc_slots, s0, ns,
                                                t, p->seed, p->rule, p->until_converged, st, nullptr, F, fstride),
                               "phase kernel");
                    H->hot_launches++;
                }
            return SG_OK;
        };
        if (!p->until_converged) {
            sg_status e = sweeps(0, p->max_sweeps);
            if (e != SG_OK) return e;
            T = p->max_sweeps;
        } else {
            int seg = 2;
            uint32_t hflag = 0;
            while (T < p->max_sweeps) {
                const int k = std::min(seg, p->max_sweeps - T);
                sg_status e = sweeps(T, T + k);
                if (e != SG_OK) return e;
                T += k;
                if (T >= p->max_sweeps) break;
                SG_HIP(sg::launch_fill_u32(flag, 1, 0u, st), "fill kernel");
                SG_HIP(sg::launch_any_active(rs, q.R, T, flag, st), "activity kernel");
                CopiesOut out(H);
                SG_HIP(out.copy(&hflag, flag, 4, st), "flag copy");
                SG_HIP(hipStreamSynchronize(st), "stream sync");
                out.finish();
                if (!hflag) break;
                seg = std::min(seg * 2, 64);
            }
        }
        if (qi == which.back()) SG_HIP(hipEventRecord(H->evh1, st), "event record");
        SG_HIP(sg::launch_end(rs, q.R, acc, q.acc_slots, T, p->until_converged, q.n, cs, st), "end kernel");
    }
    return SG_OK;
}

// ---------------------------------------------------------------------------
// graph schedule: the per-phase launches of `seg` sweeps recorded once in a
// HIP graph (on a private capture stream) and replayed on the bound stream;
// a last node advances the device sweep base the phase kernels add to their
// recorded local sweep index.

sg_status run_graph_schedule(sg_handle H, const sg_run_params* p, const std::vector<int>& which)
{
    hipStream_t st = H->stream;
    sg::CallStats* cs = H->at<sg::CallStats>(H->off_stats);
    uint32_t* flag = H->at<uint32_t>(H->off_flag);
    if (!H->cap_stream) SG_HIP(hipStreamCreateWithFlags(&H->cap_stream, hipStreamNonBlocking), "stream create");
    for (int qi : which) {
        const HostInst& q = H->insts[qi];
        const sg::InstDev I = H->view(q);
        sg::RepState* rs = H->reps() + q.rep_base;
        int8_t* spins = H->at<int8_t>(q.off_spins);
        int64_t* acc = H->at<int64_t>(q.off_acc);
        int32_t* tb = H->at<int32_t>(H->off_tbase) + qi;
        const sg::WideDev W = q.wide ? H->wview(q) : sg::WideDev{};
        SG_HIP(sg::launch_begin(rs, q.R, acc, (int64_t)q.R * q.acc_slots * 2, st), "begin kernel");
        SG_HIP(sg::launch_fill_u32(tb, 1, 0u, st), "fill kernel");
        const int seg = std::max(1, std::min(H->graph_sweeps, p->max_sweeps));
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        auto cleanup = [&]() {
            if (exec) {
                (void)hipStreamSynchronize(st);  // no replay may still be queued
                (void)hipGraphExecDestroy(exec);
            }
            if (graph) (void)hipGraphDestroy(graph);
            exec = nullptr;
            graph = nullptr;
        };
        if (p->max_sweeps > 0) {
            SG_HIP(hipStreamBeginCapture(H->cap_stream, hipStreamCaptureModeRelaxed), "graph capture");
            hipError_t ce = hipSuccess;
            for (int t = 0; t < seg && ce == hipSuccess; ++t)
                for (int32_t c = 0; c < q.C && ce == hipSuccess; ++c) {
                    const int s0 = q.colour_slice[c], ns = q.colour_slice[c + 1] - s0;
                    ce = q.wide ? sg::launch_wide_phase(W, spins, (int64_t)q.spin_stride, rs, q.R, acc, q.acc_slots,
                                                        s0, ns, t, p->seed, p->rule, p->until_converged,
                                                        H->cap_stream, tb)
                                : sg::launch_phase(I, spins, (int64_t)q.spin_stride, rs, q.R, acc, q.acc_slots, s0,
                                                   ns, t, p->seed, p->rule, p->until_converged, H->cap_stream, tb);
                }
            if (ce == hipSuccess) ce = sg::launch_bump(tb, seg, H->cap_stream);
            hipError_t ee = hipStreamEndCapture(H->cap_stream, &graph);
            if (ce != hipSuccess || ee != hipSuccess) {
                cleanup();
                return hip_fail(ce != hipSuccess ? ce : ee, "graph capture");
            }
            hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            if (ie != hipSuccess) {
                cleanup();
                return hip_fail(ie, "graph instantiate");
            }
        }
        if (qi == which.front()) {
            SG_HIP(hipEventRecord(H->evh0, st), "event record");
            H->hot_launches = 0;
        }
        int T = 0;
        bool stopped = false;
        while (!stopped && T + seg <= p->max_sweeps) {
            hipError_t le = hipGraphLaunch(exec, st);
            if (le != hipSuccess) {
                cleanup();
                return hip_fail(le, "graph launch");
            }
            H->hot_launches += seg * q.C;
            T += seg;
            if (p->until_converged && T < p->max_sweeps) {
                uint32_t hflag = 0;
                hipError_t e1 = sg::launch_fill_u32(flag, 1, 0u, st);
                if (e1 == hipSuccess) e1 = sg::launch_any_active(rs, q.R, T, flag, st);
                CopiesOut out(H);
                if (e1 == hipSuccess) e1 = out.copy(&hflag, flag, 4, st);
                if (e1 == hipSuccess) e1 = hipStreamSynchronize(st);
                if (e1 != hipSuccess) {
                    cleanup();
                    return hip_fail(e1, "activity check");
                }
                out.finish();
                stopped = hflag == 0;
            }
        }
        cleanup();
        // fewer than a segment left: plain launches at absolute sweep indices
        for (; !stopped && T < p->max_sweeps; ++T)
            for (int32_t c = 0; c < q.C; ++c) {
                const int s0 = q.colour_slice[c], ns = q.colour_slice[c + 1] - s0;
                if (q.wide)
                    SG_HIP(sg::launch_wide_phase(W, spins, (int64_t)q.spin_stride, rs, q.R, acc, q.acc_slots, s0, ns,
                                                 T, p->seed, p->rule, p->until_converged, st),
                           "wide phase kernel");
                else
                    SG_HIP(sg::launch_phase(I, spins, (int64_t)q.spin_stride, rs, q.R, acc, q.acc_slots, s0, ns, T,
                                            p->seed, p->rule, p->until_converged, st),
                           "phase kernel");
                H->hot_launches++;
            }
        if (qi == which.back()) SG_HIP(hipEventRecord(H->evh1, st), "event record");
        SG_HIP(sg::launch_end(rs, q.R, acc, q.acc_slots, T, p->until_converged, q.n, cs, st), "end kernel");
    }
    return SG_OK;
}

// ---------------------------------------------------------------------------
// lattice schedules: whole lattice per workgroup, or co-resident tiles

bool lattice_wg_fits(const sg_ctx* H, const HostInst& q) { return q.n <= H->lattice_wg_max_n; }

// Largest tiling whose boxes fit LDS and whose workgroups are co-resident:
// minimise the largest box (work per workgroup per phase).
bool choose_tiling(const sg_ctx* H, const HostInst& q, sg::TileGeom& tg)
{
    const int k = std::max(1, H->lattice_k);
    int cap_limit = kMaxLatticeTiles;
    if (H->lattice_max_tiles > 0) cap_limit = std::min(cap_limit, H->lattice_max_tiles);
    std::vector<std::pair<size_t, int>> cap_cache;  // LDS bytes -> co-resident workgroups
    auto cap_for = [&](const sg::TileGeom& g) {
        const size_t lds = sg::lattice_tiles_lds(g, q.lat_L, q.lat_D);
        for (auto& c : cap_cache)
            if (c.first == lds) return c.second;
        const int c = sg::lattice_tiles_max_blocks(g, q.lat_L, q.lat_D);
        cap_cache.emplace_back(lds, c);
        return c;
    };
    bool found = false;
    int64_t bestV = INT64_MAX;
    int bestT = 0;
    const int a0 = q.lat_D == 2 ? 1 : 0;
    for (int p0 = 1; p0 <= (a0 ? 1 : q.lat_L[0] / k); ++p0)
        for (int p1 = 1; p1 <= q.lat_L[1] / k; ++p1)
            for (int p2 = 1; p2 <= q.lat_L[2] / k; ++p2) {
                const int T = p0 * p1 * p2;
                if (T > cap_limit) break;
                sg::TileGeom g{};
                g.P[0] = p0; g.P[1] = p1; g.P[2] = p2; g.k = k;
                int64_t V = 1;
                for (int a = 0; a < 3; ++a)
                    V *= (q.lat_L[a] + g.P[a] - 1) / g.P[a] + ((a < a0) ? 0 : 2 * k);
                if (!(V < bestV || (V == bestV && T < bestT))) continue;
                if (sg::lattice_tiles_ns(g, q.lat_L, q.lat_D) == 0) continue;
                if ((q.lat_L[2] + p2 - 1) / p2 > 32) continue;  // an interior z-row is one 32-bit word
                if (q.lat_L[2] / p2 < 4) continue;               // keeps the exchange within its allocation
                if ((int64_t)sg::lattice_tiles_words(g, q.lat_L) * 16 * q.R > (int64_t)q.lat_g_bytes) continue;
                if ((int64_t)T * q.R > cap_for(g)) continue;
                bestV = V;
                bestT = T;
                tg = g;
                found = true;
            }
    return found;
}

// Tiling and halo width of the bit-plane kernel.  Per colour phase a tile
// costs a fixed latency plus one step per wavefront that each SIMD runs over
// the rows deeper than the phase index (64 rows per wavefront, four SIMDs per
// compute unit; under GREEDY_TIE a step also holds the wavefront's tie draws),
// and every k phases an exchange (a fixed latency, plus a pass per further
// 1024 box rows).  The constants are microseconds fitted to the measured time
// of 1000 sweeps of this kernel on the 10^6-spin lattice over 31 tilings and
// halo widths under both rules; the choice minimises the cost per phase,
// subject to LDS, co-residency and the geometry limits of the kernel.
bool choose_tiling_msc(const sg_ctx* H, const HostInst& q, bool tie, sg::TileGeom& tg, double* model_phase_us = nullptr,
                       double* model_exchange_us = nullptr)
{
    int cap_limit = kMaxLatticeTiles;
    if (H->lattice_max_tiles > 0) cap_limit = std::min(cap_limit, H->lattice_max_tiles);
    std::vector<std::pair<size_t, int>> cap_cache;
    auto cap_for = [&](const sg::TileGeom& g) {
        const size_t lds = sg::lattice_msc_lds(g, q.lat_L, q.lat_D);
        for (auto& c : cap_cache)
            if (c.first == lds) return c.second;
        const int c = sg::lattice_msc_max_blocks(g, q.lat_L, q.lat_D);
        cap_cache.emplace_back(lds, c);
        return c;
    };
    const int a0 = q.lat_D == 2 ? 1 : 0;
    const int k_lo = H->msc_k ? H->msc_k : 1, k_hi = H->msc_k ? H->msc_k : 62;
    bool found = false;
    double best = 1e300;
    int bestT = 0;
    for (int p0 = 1; p0 <= (a0 ? 1 : q.lat_L[0]) && p0 <= cap_limit; ++p0)
        for (int p1 = 1; p1 <= q.lat_L[1] && p0 * p1 <= cap_limit; ++p1)
            for (int p2 = 1; p2 <= q.lat_L[2]; ++p2) {
                const int T = p0 * p1 * p2;
                if (T > cap_limit) break;
                if (q.lat_L[2] / p2 < 4) continue;  // keeps the exchange within its allocation
                for (int k = k_lo; k <= k_hi; ++k) {
                    sg::TileGeom g{};
                    g.P[0] = p0; g.P[1] = p1; g.P[2] = p2; g.k = k;
                    if (!sg::lattice_msc_geometry_ok(g, q.lat_L, q.lat_D)) continue;
                    if (sg::lattice_msc_lds(g, q.lat_L, q.lat_D) > kLatLdsBudget) continue;
                    int B[3];
                    for (int a = 0; a < 3; ++a)
                        B[a] = (q.lat_L[a] + g.P[a] - 1) / g.P[a] + ((a < a0) ? 0 : 2 * k);
                    const double rows = (double)B[0] * B[1];
                    const double ex0 = tie ? 2.0 : 2.1, ex1 = 0.4;
                    const double ph0 = tie ? 0.84 : 0.19, ph1 = tie ? 0.49 : 0.28;
                    const double excost = ex0 + ex1 * (std::ceil(rows / 1024.0) - 1.0);
                    double cost = excost;
                    for (int qq = 0; qq < k; ++qq) {
                        const double ax = a0 ? 1.0 : std::max(0, B[0] - 2 * (qq + 1));
                        const double ay = std::max(0, B[1] - 2 * (qq + 1));
                        const double steps = std::ceil(std::ceil(ax * ay / 64.0) / 4.0);
                        cost += ph0 + ph1 * steps;
                    }
                    cost /= k;
                    if (!(cost < best - 1e-9 || (std::fabs(cost - best) <= 1e-9 && T < bestT))) continue;
                    if ((int64_t)sg::lattice_tiles_words(g, q.lat_L) * 16 * q.R > (int64_t)q.lat_g_bytes) continue;
                    if ((int64_t)T * q.R > cap_for(g)) continue;
                    best = cost;
                    bestT = T;
                    tg = g;
                    found = true;
                    if (model_phase_us) *model_phase_us = (cost * k - excost) / k;
                    if (model_exchange_us) *model_exchange_us = excost;
                }
            }
    return found;
}

// The tiling of a lattice instance for the tile kernels (the bit-plane kernel
// when it applies and fits, else the byte kernel); it depends only on the
// instance, the rule and the knobs, so it is searched once per setting.
// False when no tiling fits.
bool lattice_tiling(const sg_ctx* H, const HostInst& q, int rule, sg::TileGeom& tg, bool& msc)
{
    const std::array<int32_t, 6> key{{rule, H->lattice_msc, H->msc_k, H->lattice_max_tiles, H->lattice_k, 1}};
    if (q.tile_key != key) {
        sg::TileGeom g{};
        double mph = 0.0, mex = 0.0;
        const bool m = q.lat_msc && H->lattice_msc && choose_tiling_msc(H, q, rule == 1, g, &mph, &mex);
        const bool found = m || choose_tiling(H, q, g);
        q.tile_key = key;
        q.tile_geom = g;
        q.tile_msc = m ? 1 : 0;
        q.tile_found = found ? 1 : 0;
        q.tile_model_phase_us = m ? mph : 0.0;
        q.tile_model_ex_us = m ? mex : 0.0;
    }
    tg = q.tile_geom;
    msc = q.tile_msc != 0;
    return q.tile_found != 0;
}

sg_status run_lattice_schedule(sg_handle H, const sg_run_params* p, const std::vector<int>& which)
{
    hipStream_t st = H->stream;
    sg::CallStats* cs = H->at<sg::CallStats>(H->off_stats);
    uint32_t* err = H->at<uint32_t>(H->off_err);
    // the tile kernels' error flag: cleared once per call (so a failed wait in
    // any launch of the call is reported), read with the call totals at its end
    SG_HIP(sg::launch_fill_u32(err, 1, 0u, st), "fill kernel");
    H->lat_err_check = true;
    for (int qi : which) {
        const HostInst& q = H->insts[qi];
        sg::RepState* rs = H->reps() + q.rep_base;
        int8_t* spins = H->at<int8_t>(q.off_spins);
        int64_t* acc = H->at<int64_t>(q.off_acc);
        const sg::LatticeDev Lt = H->lat_view(q);
        SG_HIP(sg::launch_begin(rs, q.R, acc, (int64_t)q.R * q.acc_slots * 2, st), "begin kernel");
        const int T = p->max_sweeps;
        int T_done = T;         // sweeps launched (fewer when the tile chunks stop early)
        bool absolute = false;  // the bit-plane kernel leaves final energies, not changes
        if (T > 0) {
            if (lattice_wg_fits(H, q)) {
                SG_HIP(hipEventRecord(H->evh0, st), "event record");
                SG_HIP(sg::launch_lattice_wg(Lt, spins, (int64_t)q.spin_stride, rs, q.R, acc, q.acc_slots, T, p->seed,
                                             p->rule, p->until_converged, st),
                       "lattice workgroup kernel");
                SG_HIP(hipEventRecord(H->evh1, st), "event record");
                H->hot_launches = 1;
            } else {
                sg::TileGeom tg{};
                bool msc = false;
                if (!lattice_tiling(H, q, p->rule, tg, msc))
                    return fail(SG_EINVAL, "lattice schedule: no tiling of %dx%dx%d fits", q.lat_L[0], q.lat_L[1],
                                q.lat_L[2]);
                const HostInst& qm = q;
                if (p->until_converged && !(msc && p->rule == SG_RULE_GREEDY))
                    return fail(SG_EINVAL, "lattice schedule: the stopping rule on a lattice of %d spins needs the "
                                           "bit-plane tile kernel under GREEDY", q.n);
                // exchange words (8 bytes: epoch tag and bits): at most n / (smallest z
                // extent) + one row per tile, per copy
                const int64_t words = sg::lattice_tiles_words(tg, q.lat_L) * q.R;
                if ((uint64_t)words * 16 > q.lat_g_bytes)
                    return fail(SG_ERANGE, "lattice tile exchange needs %lld bytes", (long long)(words * 16));
                // tags of a launch's epochs start at 1: clear the tags of earlier launches
                uint64_t* G0 = H->at<uint64_t>(q.off_lat_g);
                uint64_t* cnt = H->at<uint64_t>(q.off_lat_cnt);
                SG_HIP(hipEventRecord(H->evh0, st), "event record");
                H->hot_launches = 0;
                int launched = 0;  // sweeps launched in this call
                while (launched < T) {
                    // under the stopping rule the sweeps go in chunks of at most
                    // kConvChunk (one counter slot per sweep and replica), and a
                    // chunk ends early once every replica's tiles have seen a sweep
                    // without a flip
                    const int Tc = p->until_converged ? std::min(T - launched, H->conv_chunk) : T;
                    SG_HIP(sg::launch_fill_u32(reinterpret_cast<uint32_t*>(G0), (uint64_t)words * 4, 0u, st),
                           "fill kernel");
                    if (p->until_converged)
                        SG_HIP(sg::launch_fill_u32(reinterpret_cast<uint32_t*>(cnt), (uint64_t)q.R * Tc * 2, 0u, st),
                               "fill kernel");
                    if (msc)
                        SG_HIP(sg::launch_lattice_msc(Lt, tg, spins, (int64_t)q.spin_stride, G0, G0 + words, err, rs,
                                                      q.R, acc, q.acc_slots, Tc, p->seed, p->rule, st,
                                                      p->until_converged ? cnt : nullptr, launched),
                               "lattice bit-plane kernel");
                    else
                        SG_HIP(sg::launch_lattice_tiles(Lt, tg, spins, (int64_t)q.spin_stride, G0, G0 + words, err,
                                                        rs, q.R, acc, q.acc_slots, Tc, p->seed, p->rule, st),
                               "lattice tile kernel");
                    H->hot_launches++;
                    launched += Tc;
                    if (!p->until_converged || launched >= T) break;
                    uint32_t* flag = H->at<uint32_t>(H->off_flag);
                    uint32_t hflag = 0;
                    SG_HIP(sg::launch_fill_u32(flag, 1, 0u, st), "fill kernel");
                    SG_HIP(sg::launch_any_active(rs, q.R, launched, flag, st), "activity kernel");
                    CopiesOut out(H);
                    SG_HIP(out.copy(&hflag, flag, 4, st), "flag copy");
                    SG_HIP(hipStreamSynchronize(st), "stream sync");
                    out.finish();
                    if (!hflag) break;
                }
                T_done = launched;
                H->last_msc = msc ? 1 : 0;
                absolute = msc;
                if (msc) H->e_written[(size_t)qi] = 1;
                SG_HIP(hipEventRecord(H->evh1, st), "event record");
                H->last_tiles[0] = tg.P[0];
                H->last_tiles[1] = tg.P[1];
                H->last_tiles[2] = tg.P[2];
                H->last_tiles[3] = tg.k;
                // the tiling cost model's prediction of this launch: C colour
                // phases per sweep, one exchange every k phases
                const double phases = (double)T * q.C;
                H->last_model_phase_us = msc ? qm.tile_model_phase_us : 0.0;
                H->last_model_ex_us = msc ? qm.tile_model_ex_us : 0.0;
                H->last_model_exchanges = msc ? (int64_t)std::ceil(phases / tg.k) : 0;
                H->last_model_phases = msc ? (int64_t)phases : 0;
            }
        }
        SG_HIP(sg::launch_end(rs, q.R, acc, q.acc_slots, T_done, p->until_converged, q.n, cs, st, absolute),
               "end kernel");
    }
    return SG_OK;
}

// ---------------------------------------------------------------------------
// batched schedules

constexpr size_t kLdsBudget = 160 * 1024 - 6 * 1024;  // dynamic LDS left beside the kernels' static arrays
constexpr int32_t kQueueMaxN = 150000;                  // largest item of the queue schedule (spins in LDS)
constexpr int32_t kBlockGroupsAuto = 4;                 // most restart groups per block workgroup (auto)

// Restarts per block workgroup for instance q (0 if the block schedule cannot
// hold it).  Default 64: smaller workgroups fit more per CU and keep one
// launch for a batch (measured on 4096 Chimera instances x 256 restarts:
// 9.6 ms at 64, 15.2 ms at 128, 15.8 ms with the largest size that fits).
int block_rg_for(const sg_ctx* H, const HostInst& q)
{
    if (q.wide) return 0;
    const int want = H->block_rg ? H->block_rg : 64;
    for (int rg = want; rg >= 64; rg -= 64) {
        if (H->block_rg && rg != H->block_rg) break;
        if (rg != 64 && rg != 128 && rg != 192 && rg != 256) continue;
        if (16 % (rg / 64)) continue;
        const size_t lds = sg::block_lds_bytes(q.n, (int)q.nbr.size(), (int)q.ta.size(), (int)q.slices.size(), q.C, rg);
        if (lds <= kLdsBudget) return rg;
    }
    return 0;
}

// Groups of 32 restarts per bit-sliced workgroup for instance q: enough for
// its restarts, at most bits_groups (8 measured fastest on 4096 Chimera
// instances x 256 restarts: 4.3 ms, against 5.5 ms with 4 or 16).
int bits_ng_for(const sg_ctx* H, const HostInst& q)
{
    int ng = 2;
    while (ng < H->bits_groups && ng * 32 < q.R) ng *= 2;
    return ng;
}

// LDS of the bit-sliced block kernel for instance q (0 if it does not apply).
size_t bits_lds_for(const sg_ctx* H, const HostInst& q)
{
    if (!q.bits_ok) return 0;
    const size_t lds = sg::block_bits_lds_bytes(q.n, (int)q.nbr.size(), (int)q.ta.size(), (int)q.slices.size(), q.C,
                                                bits_ng_for(H, q));
    return lds <= kLdsBudget ? lds : 0;
}

sg_status run_block_bits_ng(sg_handle H, const sg_run_params* p, const std::vector<int>& which, int NG);

// GREEDY on the bit-sliced block kernel: one workgroup per range of restarts
// (up to four workgroup-fulls of groups of 32, taken in turn as groups stop);
// a finished group computes its restarts' energies from their final spins.
sg_status run_block_bits(sg_handle H, const sg_run_params* p, const std::vector<int>& which_all)
{
    // one launch per group count (a template parameter of the kernel)
    std::vector<int> ngs;
    for (int qi : which_all) {
        const int ng = bits_ng_for(H, H->insts[qi]);
        if (std::find(ngs.begin(), ngs.end(), ng) == ngs.end()) ngs.push_back(ng);
    }
    for (int NG : ngs) {
        std::vector<int> which;
        for (int qi : which_all)
            if (bits_ng_for(H, H->insts[qi]) == NG) which.push_back(qi);
        sg_status e = run_block_bits_ng(H, p, which, NG);
        if (e != SG_OK) return e;
    }
    return SG_OK;
}

sg_status run_block_bits_ng(sg_handle H, const sg_run_params* p, const std::vector<int>& which, int NG)
{
    hipStream_t st = H->stream;
    size_t lds = 0;
    int64_t groups = 0;
    for (int qi : which) {
        const HostInst& q = H->insts[qi];
        lds = std::max(lds, bits_lds_for(H, q));
        groups += (q.R + 31) / 32;
    }
    int m = H->block_groups;
    if (m <= 0) {
        const int cap = std::max(1, sg::block_bits_max_blocks(lds, NG));
        m = (int)std::max<int64_t>(1, std::min<int64_t>(kBlockGroupsAuto, groups / ((int64_t)NG * cap)));
    }
    H->h_bitems.clear();
    for (int qi : which) {
        const HostInst& q = H->insts[qi];
        for (int r0 = 0; r0 < q.R; r0 += 32 * NG * m)
            H->h_bitems.push_back(sg::BlockItem{qi, r0, std::min(32 * NG * m, q.R - r0), 0});
    }
    if ((int64_t)H->h_bitems.size() > H->n_block_item_cap)
        return fail(SG_EINVAL, "block schedule: item list exceeds its allocation");
    sg::BlockItem* dit = H->at<sg::BlockItem>(H->off_bitems);
    SG_HIP(hipMemcpyAsync(dit, H->h_bitems.data(), H->h_bitems.size() * sizeof(sg::BlockItem), hipMemcpyHostToDevice,
                          st),
           "upload block items");
    SG_HIP(hipEventRecord(H->evh0, st), "event record");
    SG_HIP(sg::launch_block_bits(H->at<sg::InstTab>(H->off_tab), H->at<int32_t>(H->off_ctab), dit,
                                 (int)H->h_bitems.size(), lds, H->reps(), H->at<sg::CallStats>(H->off_stats), NG,
                                 p->max_sweeps, p->until_converged, st),
           "bit-sliced block kernel");
    SG_HIP(hipEventRecord(H->evh1, st), "event record");
    H->hot_launches = 1;
    H->last_bits = 1;
    SG_HIP(hipStreamSynchronize(st), "stream sync");  // the host item lists are reused
    return SG_OK;
}

// The block schedule runs this instance on the bit-sliced kernel.
bool bits_path(const sg_ctx* H, const sg_run_params* p, const HostInst& q)
{
    return H->block_bits && p->rule == SG_RULE_GREEDY && p->max_sweeps > 0 && bits_lds_for(H, q) > 0;
}

sg_status run_block_schedule(sg_handle H, const sg_run_params* p, const std::vector<int>& which_all)
{
    if (which_all.empty()) return SG_OK;
    hipStream_t st = H->stream;
    H->last_bits = 0;
    std::vector<int> bits, which;
    for (int qi : which_all) (bits_path(H, p, H->insts[qi]) ? bits : which).push_back(qi);
    if (!bits.empty()) {
        sg_status e = run_block_bits(H, p, bits);
        if (e != SG_OK) return e;
    }
    if (which.empty()) return SG_OK;
    // one launch per distinct restart-group size (the kernel takes it as a parameter)
    std::vector<int> rgs;
    for (int qi : which) {
        const int rg = block_rg_for(H, H->insts[qi]);
        if (std::find(rgs.begin(), rgs.end(), rg) == rgs.end()) rgs.push_back(rg);
    }
    uint64_t item_off = 0;
    for (int rg : rgs) {
        H->h_bitems.clear();
        size_t lds = 0;
        int64_t groups = 0;
        for (int qi : which) {
            const HostInst& q = H->insts[qi];
            if (block_rg_for(H, q) != rg) continue;
            groups += (q.R + rg - 1) / rg;
            lds = std::max(lds, sg::block_lds_bytes(q.n, (int)q.nbr.size(), (int)q.ta.size(), (int)q.slices.size(),
                                                    q.C, rg));
        }
        // restarts per workgroup: up to block_groups slot-fulls, which its
        // slots work through as replicas stop, while the workgroups still
        // fill the GPU
        int m = H->block_groups;
        if (m <= 0) {
            const int cap = std::max(1, sg::block_max_blocks(lds));
            m = (int)std::max<int64_t>(1, std::min<int64_t>(kBlockGroupsAuto, groups / cap));
        }
        for (int qi : which) {
            const HostInst& q = H->insts[qi];
            if (block_rg_for(H, q) != rg) continue;
            for (int r0 = 0; r0 < q.R; r0 += rg * m) {
                sg::BlockItem it{};
                it.inst = qi;
                it.r0 = r0;
                it.nr = std::min(rg * m, q.R - r0);
                H->h_bitems.push_back(it);
            }
        }
        sg::BlockItem* dit = H->at<sg::BlockItem>(H->off_bitems) + item_off;
        SG_HIP(hipMemcpyAsync(dit, H->h_bitems.data(), H->h_bitems.size() * sizeof(sg::BlockItem),
                              hipMemcpyHostToDevice, st),
               "upload block items");
        SG_HIP(hipEventRecord(H->evh0, st), "event record");
        SG_HIP(sg::launch_block(H->at<sg::InstTab>(H->off_tab), H->at<int32_t>(H->off_ctab), dit,
                                (int)H->h_bitems.size(), lds, H->reps(), H->at<sg::CallStats>(H->off_stats), rg,
                                p->max_sweeps, p->seed, p->rule, p->until_converged, st),
               "block kernel");
        SG_HIP(hipEventRecord(H->evh1, st), "event record");
        H->hot_launches = 1;
        SG_HIP(hipStreamSynchronize(st), "stream sync");  // the host item list is reused
        item_off += H->h_bitems.size();
    }
    return SG_OK;
}

sg_status run_queue_schedule(sg_handle H, const sg_run_params* p, const std::vector<int>& which)
{
    if (which.empty()) return SG_OK;
    hipStream_t st = H->stream;
    // items sorted by decreasing size (longest first), large items before wavefront items
    H->h_qitems.clear();
    int nmax_big = 0, nmax_small = 0;
    for (int qi : which)
        for (int r = 0; r < H->insts[qi].R; ++r) H->h_qitems.push_back(sg::QueueItem{qi, r});
    std::stable_sort(H->h_qitems.begin(), H->h_qitems.end(), [&](const sg::QueueItem& a, const sg::QueueItem& b) {
        return H->insts[a.inst].n > H->insts[b.inst].n;
    });
    int n_big = 0;
    for (const sg::QueueItem& it : H->h_qitems) {
        const int n = H->insts[it.inst].n;
        if (n > H->queue_wave_max_n) {
            ++n_big;
            nmax_big = std::max(nmax_big, n);
        } else {
            nmax_small = std::max(nmax_small, n);
        }
    }
    const int wave_lds = (nmax_small + 15) / 16 * 16;
    size_t lds = std::max<size_t>((size_t)nmax_big, (size_t)wave_lds * 16);
    lds = std::max<size_t>((lds + 15) / 16 * 16, 16);
    if (lds > kLdsBudget) return fail(SG_EINVAL, "queue schedule: an item needs %zu bytes of LDS", lds);
    int grid = H->queue_grid;
    if (grid <= 0) grid = sg::queue_max_blocks(lds);
    if (grid <= 0) grid = 256;
    grid = std::min<int>(grid, (int)H->h_qitems.size());
    uint32_t* cnt = H->at<uint32_t>(H->off_qcnt);
    SG_HIP(sg::launch_fill_u32(cnt, 2, 0u, st), "fill kernel");
    sg::QueueItem* dit = H->at<sg::QueueItem>(H->off_qitems);
    SG_HIP(hipMemcpyAsync(dit, H->h_qitems.data(), H->h_qitems.size() * sizeof(sg::QueueItem), hipMemcpyHostToDevice,
                          st),
           "upload queue items");
    SG_HIP(hipEventRecord(H->evh0, st), "event record");
    H->hot_launches = 1;
    SG_HIP(sg::launch_queue(H->at<sg::InstTab>(H->off_tab), H->at<int32_t>(H->off_ctab), dit, n_big,
                            (int)H->h_qitems.size(), cnt, wave_lds, lds, grid, H->reps(),
                            H->at<sg::CallStats>(H->off_stats), p->max_sweeps, p->seed, p->rule, p->until_converged,
                            st),
           "queue kernel");
    SG_HIP(hipEventRecord(H->evh1, st), "event record");
    SG_HIP(hipStreamSynchronize(st), "stream sync");  // the host item list is reused
    H->last_queue_grid = grid;
    return SG_OK;
}

// ---------------------------------------------------------------------------
// schedule choice

bool can_lattice(const sg_ctx* H, const HostInst& q, const sg_run_params* p)
{
    if (!q.lat_ok) return false;
    if (lattice_wg_fits(H, q) || !p->until_converged) return true;
    // the stopping rule on the tile kernels: the bit-plane kernel under GREEDY,
    // where a sweep without a flip is a fixed point (later sweeps change nothing)
    if (p->rule != SG_RULE_GREEDY) return false;
    sg::TileGeom tg{};
    bool msc = false;
    return lattice_tiling(H, q, p->rule, tg, msc) && msc;
}
bool can_block(const sg_ctx* H, const HostInst& q) { return block_rg_for(H, q) > 0; }
bool can_queue(const HostInst& q) { return !q.wide && q.n <= kQueueMaxN; }

// Per-instance schedule, or -1 when the requested schedule cannot run some instance.
int assign_schedules(const sg_ctx* H, const sg_run_params* p, std::vector<int>& out)
{
    out.assign(H->insts.size(), SG_SCHED_PHASE);
    const int req = p->schedule;
    int64_t queue_items = 0;
    for (const HostInst& q : H->insts)
        if (!q.lat_ok && can_queue(q) && !(q.R >= H->block_min_restarts && can_block(H, q))) queue_items += q.R;
    for (size_t k = 0; k < H->insts.size(); ++k) {
        const HostInst& q = H->insts[k];
        int s;
        switch (req) {
        case SG_SCHED_AUTO:
            if (can_lattice(H, q, p)) s = SG_SCHED_LATTICE;
            else if (q.R >= H->block_min_restarts && can_block(H, q)) s = SG_SCHED_BLOCK;
            else if (can_queue(q) && queue_items >= H->queue_min_items) s = SG_SCHED_QUEUE;
            else if (H->fields_ws && !q.wide) s = SG_SCHED_FIELDS;
            else s = H->auto_graph ? SG_SCHED_GRAPH : SG_SCHED_PHASE;
            break;
        case SG_SCHED_PHASE: s = SG_SCHED_PHASE; break;
        case SG_SCHED_GRAPH: s = SG_SCHED_GRAPH; break;
        case SG_SCHED_FIELDS: s = H->fields_ws && !q.wide ? SG_SCHED_FIELDS : -1; break;
        case SG_SCHED_LATTICE: s = can_lattice(H, q, p) ? SG_SCHED_LATTICE : -1; break;
        case SG_SCHED_BLOCK: s = can_block(H, q) ? SG_SCHED_BLOCK : -1; break;
        case SG_SCHED_QUEUE: s = can_queue(q) ? SG_SCHED_QUEUE : -1; break;
        default: s = -1;
        }
        if (s < 0) return -1;
        out[k] = s;
    }
    int first = out.empty() ? SG_SCHED_PHASE : out[0];
    for (int s : out)
        if (s != first) return SG_SCHED_AUTO;  // mixed
    return first;
}

// Dense hyper-Ising handles: sweeps or passes, one lane per replica.
sg_status run_dense(sg_handle H, const sg_run_params* p, sg_run_stats* stats)
{
    if (p->schedule != SG_SCHED_AUTO && p->schedule != SG_SCHED_DENSE)
        return fail(SG_EINVAL, "a dense handle runs under SG_SCHED_AUTO or SG_SCHED_DENSE only");
    hipStream_t st = H->stream;
    SG_HIP(sg::launch_fill_u32(H->at<uint32_t>(H->off_stats), sizeof(sg::CallStats) / 4, 0u, st), "fill kernel");
    SG_HIP(hipEventRecord(H->ev0, st), "event record");
    SG_HIP(hipEventRecord(H->evh0, st), "event record");
    if (p->max_sweeps > 0)
        SG_HIP(sg::launch_dense_run(H->at<sg::DenseTab>(H->off_dtab), H->at<sg::BlockItem>(H->off_ditems),
                                    (int)H->h_ditems.size(), H->dense_nmax, H->reps(),
                                    H->at<sg::CallStats>(H->off_stats), p->rule, p->max_sweeps, p->until_converged,
                                    p->seed, st),
               "dense kernel");
    SG_HIP(hipEventRecord(H->evh1, st), "event record");
    SG_HIP(hipEventRecord(H->ev1, st), "event record");
    H->hot_launches = p->max_sweeps > 0 ? 1 : 0;
    sg::CallStats cs;
    SG_HIP(hipMemcpyAsync(&cs, H->at<sg::CallStats>(H->off_stats), sizeof cs, hipMemcpyDeviceToHost, st), "stats copy");
    SG_HIP(hipStreamSynchronize(st), "stream sync");
    float ms = 0.f, hms = 0.f;
    SG_HIP(hipEventElapsedTime(&ms, H->ev0, H->ev1), "event time");
    H->hot_us = hipEventElapsedTime(&hms, H->evh0, H->evh1) == hipSuccess ? hms * 1000.0 : 0.0;
    if (stats) {
        stats->attempts = (int64_t)cs.attempts;
        stats->flips = (int64_t)cs.flips;
        stats->sweeps_max = (int64_t)cs.sweeps_max;
        stats->n_unconverged = (int32_t)cs.unconverged;
        stats->schedule_used = SG_SCHED_DENSE;
        stats->kernel_ms = ms;
    }
    if (p->until_converged && cs.unconverged)
        return fail(SG_ENOTCONV, "%llu replicas did not converge within %d %s", (unsigned long long)cs.unconverged,
                    p->max_sweeps, p->rule == SG_RULE_FM ? "passes" : "sweeps");
    return SG_OK;
}

// The pass-based search (SG_RULE_FM): every replica of every instance is one
// wavefront item, largest instances first.
sg_status run_fm(sg_handle H, const sg_run_params* p, sg_run_stats* stats)
{
    if (p->schedule != SG_SCHED_AUTO && p->schedule != SG_SCHED_FM)
        return fail(SG_EINVAL, "rule SG_RULE_FM runs under SG_SCHED_AUTO or SG_SCHED_FM only");
    int nmax = 1, lnmax = 1;
    bool tri = false, key32 = true;
    int64_t lane_reps = 0, wave_reps = 0;
    auto on_lanes = [&](const HostInst& q) { return H->fm_lanes && q.fml_off != UINT64_MAX; };
    int64_t big_reps = 0;
    for (const HostInst& q : H->insts) {
        if (q.n > kFmMaxN) {
            if (q.off_fmb_rows == UINT64_MAX)
                return fail(SG_EINVAL,
                            "rule SG_RULE_FM: instance %zu has %d spins (more than %d): its pass kernel needs "
                            "fm_slots > 0 set before sg_bind and at most %d spins",
                            (size_t)(&q - H->insts.data()), q.n, kFmMaxN, kFmBigMaxN);
            big_reps += q.R;
            continue;
        }
        if (q.wide) continue;  // a launch of its own below
        if (on_lanes(q)) {
            lnmax = std::max(lnmax, q.n);
            lane_reps += q.R;
            continue;
        }
        wave_reps += q.R;
        nmax = std::max(nmax, q.n);
        tri = tri || q.t > 0;
        // 32-bit move keys: every gain |2 s f| < 2^19 and external indices below 4096
        key32 = key32 && 2 * q.max_w < (int64_t)1 << 19 && q.n <= 4096 && H->fm_key32;
    }
    H->last_key32 = wave_reps && key32 ? 1 : 0;
    H->last_fm_lanes = (int32_t)std::min<int64_t>(lane_reps, INT32_MAX);
    hipStream_t st = H->stream;
    H->h_qitems.clear();
    for (size_t k = 0; k < H->insts.size(); ++k)
        if (!on_lanes(H->insts[k]) && !H->insts[k].wide && H->insts[k].n <= kFmMaxN)
            for (int32_t r = 0; r < H->insts[k].R; ++r) H->h_qitems.push_back(sg::QueueItem{(int32_t)k, r});
    std::stable_sort(H->h_qitems.begin(), H->h_qitems.end(), [&](const sg::QueueItem& a, const sg::QueueItem& b) {
        return H->insts[a.inst].n > H->insts[b.inst].n;
    });
    // lane kernel items: restarts [r0, r0 + nr) of one instance per wavefront,
    // nr the largest multiple of 64 that still gives every resident wavefront
    // an item (a wavefront refills its lanes from its own item as replicas
    // finish, so longer items lose less to the replicas' uneven pass counts)
    H->h_fmitems.clear();
    int32_t nr = 64, lw = 1;
    if (lane_reps) {
        // a workgroup of W wavefronts shares its item: restarts in multiples of 64 W
        lw = std::max(1, sg::fml_waves_per_block(lnmax, H->fm_lane_waves));
        const int32_t unit = 64 * lw;
        int32_t dc = 4, tt = 0;
        for (const HostInst& q : H->insts)
            if (on_lanes(q)) {
                dc = q.fml_dc;
                tt = q.fml_tt;
                break;
            }
        const int64_t resident = std::max(1, sg::fml_resident_blocks(lnmax, lw, dc, tt));
        int32_t rmax = unit;
        for (const HostInst& q : H->insts)
            if (on_lanes(q)) rmax = std::max(rmax, (q.R + unit - 1) / unit * unit);
        if (H->fm_lane_restarts) {
            nr = H->fm_lane_restarts;
        } else {
            for (int32_t c = rmax; c >= unit; c -= unit) {
                int64_t items = 0;
                for (const HostInst& q : H->insts)
                    if (on_lanes(q)) items += (q.R + c - 1) / c;
                if (items >= resident || c == unit) {
                    nr = c;
                    break;
                }
            }
        }
        for (size_t k = 0; k < H->insts.size(); ++k) {
            const HostInst& q = H->insts[k];
            if (!on_lanes(q)) continue;
            for (int32_t r0 = 0; r0 < q.R; r0 += nr)
                H->h_fmitems.push_back(sg::BlockItem{(int32_t)k, r0, std::min(nr, q.R - r0), 0});
        }
        // one launch per pair of row widths, the largest items first in each
        auto combo = [&](const sg::BlockItem& a) { return H->insts[a.inst].fml_dc * 100 + H->insts[a.inst].fml_tt; };
        std::stable_sort(H->h_fmitems.begin(), H->h_fmitems.end(), [&](const sg::BlockItem& a, const sg::BlockItem& b) {
            if (combo(a) != combo(b)) return combo(a) < combo(b);
            return (int64_t)H->insts[a.inst].n * a.nr > (int64_t)H->insts[b.inst].n * b.nr;
        });
    }
    H->last_fm_lane_nr = lane_reps ? nr : 0;
    // the wavefront-per-replica kernel: the wavefronts' slices, plus room to
    // stage one instance's structure
    size_t stage = 0;
    for (const HostInst& q : H->insts)
        if (!on_lanes(q) && !q.wide && q.n <= kFmMaxN)
            stage = std::max(stage, q.slices.size() * sizeof(sg::Slice) + q.nbr.size() * 4 + (tri ? q.ta.size() * 8 : 0));
    stage = (stage + 15) / 16 * 16;
    // wavefronts per workgroup: the most resident wavefronts per compute unit
    // (several smaller workgroups can share one), staging the instance where
    // it fits; among equals the smallest multiple of four (its wavefronts
    // spread evenly over the four SIMDs; on 4096 Chimera instances x 256
    // restarts 8 wavefronts took 1.28 s against 1.40 s with 16, the same
    // 16 resident); fm_waves bounds the count
    if (sg::fm_lds_bytes(nmax, 1) + stage > kLdsBudget) stage = 0;  // too large to stage: read from memory
    const std::array<int64_t, 5> fkey{{nmax, (int64_t)stage, tri ? 1 : 0, key32 ? 1 : 0, H->fm_waves}};
    int waves = 0;
    if (!wave_reps) {
        waves = 1;
    } else if (H->fm_key == fkey) {
        waves = H->fm_waves_cached;
    } else {
        int resident = -1;
        for (int w = 16; w >= 1; --w) {
            if (H->fm_waves && w > H->fm_waves) continue;
            const size_t lds = sg::fm_lds_bytes(nmax, w) + stage;
            if (lds > kLdsBudget) continue;
            const int r = w * sg::fm_max_blocks_per_cu(w, lds, tri, key32);
            if (r > resident || (r == resident && w % 4 == 0)) {
                resident = r;
                waves = w;
            }
        }
        if (waves > 0) {
            H->fm_key = fkey;
            H->fm_waves_cached = waves;
        }
    }
    if (waves == 0) return fail(SG_EINVAL, "rule SG_RULE_FM: no workgroup size fits LDS (fm_waves %d)", H->fm_waves);
    H->last_fm_waves = wave_reps ? waves : 0;
    sg::QueueItem* dit = H->at<sg::QueueItem>(H->off_qitems);
    uint32_t* err = H->at<uint32_t>(H->off_err);
    SG_HIP(sg::launch_fill_u32(H->at<uint32_t>(H->off_stats), sizeof(sg::CallStats) / 4, 0u, st), "fill kernel");
    SG_HIP(sg::launch_fill_u32(err, 1, 0u, st), "fill kernel");
    if (!H->h_qitems.empty())
        SG_HIP(hipMemcpyAsync(dit, H->h_qitems.data(), H->h_qitems.size() * sizeof(sg::QueueItem),
                              hipMemcpyHostToDevice, st),
               "upload items");
    if (!H->h_fmitems.empty())
        SG_HIP(hipMemcpyAsync(H->dev + H->off_fmitems, H->h_fmitems.data(), H->h_fmitems.size() * sizeof(sg::BlockItem),
                              hipMemcpyHostToDevice, st),
               "upload lane items");
    SG_HIP(hipEventRecord(H->ev0, st), "event record");
    SG_HIP(hipEventRecord(H->evh0, st), "event record");
    int lane_launches = 0;
    if (p->max_sweeps > 0)
        for (size_t a = 0; a < H->h_fmitems.size();) {
            const HostInst& q0 = H->insts[H->h_fmitems[a].inst];
            size_t b = a;
            int cn = 1;
            while (b < H->h_fmitems.size() && H->insts[H->h_fmitems[b].inst].fml_dc == q0.fml_dc &&
                   H->insts[H->h_fmitems[b].inst].fml_tt == q0.fml_tt)
                cn = std::max(cn, H->insts[H->h_fmitems[b++].inst].n);
            SG_HIP(sg::launch_fm_lanes(H->at<sg::InstTab>(H->off_tab), H->at<sg::BlockItem>(H->off_fmitems) + a,
                                       (int)(b - a), cn, lw, q0.fml_dc, q0.fml_tt, H->reps(),
                                       H->at<sg::CallStats>(H->off_stats), err, p->max_sweeps, p->until_converged, st),
                   "lane pass kernel");
            ++lane_launches;
            a = b;
        }
    if (p->max_sweeps > 0 && !H->h_qitems.empty())
        SG_HIP(sg::launch_fm(H->at<sg::InstTab>(H->off_tab), H->at<int32_t>(H->off_ctab), dit,
                             (int)H->h_qitems.size(), nmax, waves, (int)stage, tri, key32, H->reps(),
                             H->at<sg::CallStats>(H->off_stats),
                             err, p->max_sweeps, p->until_converged, st),
               "pass kernel");
    // instances in the wide form: one launch each, a wavefront per replica
    int wide_launches = 0;
    for (const HostInst& q : H->insts)
        if (q.wide && q.n <= kFmMaxN && p->max_sweeps > 0) {
            SG_HIP(sg::launch_fm_wide(H->wview(q), H->at<int8_t>(q.off_spins), (int64_t)q.spin_stride,
                                      H->reps() + q.rep_base, q.R, H->at<sg::CallStats>(H->off_stats), err,
                                      p->max_sweeps, p->until_converged, st),
                   "wide pass kernel");
            ++wide_launches;
        }
    // instances beyond a wavefront's LDS: one launch, a wavefront per slot
    int big_launches = 0;
    H->last_fm_big = 0;
    if (big_reps && p->max_sweeps > 0) {
        SG_HIP(sg::launch_fill_u32(H->at<uint32_t>(H->off_fmb_cnt), 1, 0u, st), "fill kernel");
        const int slots = (int)std::min<int64_t>(H->fm_slots, H->fmb_reps);
        SG_HIP(sg::launch_fm_big(H->at<sg::InstTab>(H->off_tab), H->at<sg::FmbRows>(H->off_fmb_ptr),
                                 H->at<sg::QueueItem>(H->off_fmb_items), (int)H->fmb_reps,
                                 H->at<uint32_t>(H->off_fmb_cnt), H->at<int32_t>(H->off_fmb_half),
                                 H->at<int32_t>(H->off_fmb_moves), H->at<uint64_t>(H->off_fmb_leaf),
                                 H->at<int8_t>(H->off_fmb_spin), H->fmb_slot_spins, H->fmb_slot_leaves, slots,
                                 (int)((H->fmb_slot_leaves + 63) / 64), H->reps(), H->at<sg::CallStats>(H->off_stats),
                                 err, p->max_sweeps, p->until_converged, st),
               "large-instance pass kernel");
        H->last_fm_big = (int32_t)std::min<int64_t>(big_reps, INT32_MAX);
        big_launches = 1;
    }
    SG_HIP(hipEventRecord(H->evh1, st), "event record");
    SG_HIP(hipEventRecord(H->ev1, st), "event record");
    H->hot_launches =
        p->max_sweeps > 0 ? lane_launches + (int)!H->h_qitems.empty() + wide_launches + big_launches : 0;
    sg::CallStats cs;
    uint32_t herr = 0;
    CopiesOut out(H);
    SG_HIP(out.copy(&cs, H->at<sg::CallStats>(H->off_stats), sizeof cs, st), "stats copy");
    SG_HIP(out.copy(&herr, err, 4, st), "error flag copy");
    SG_HIP(hipStreamSynchronize(st), "stream sync");
    out.finish();
    if (herr) return fail(SG_EDEVICE, "pass kernel: internal error (a selected move had no spin)");
    float ms = 0.f;
    SG_HIP(hipEventElapsedTime(&ms, H->ev0, H->ev1), "event time");
    float hms = 0.f;
    H->hot_us = hipEventElapsedTime(&hms, H->evh0, H->evh1) == hipSuccess ? hms * 1000.0 : 0.0;
    if (stats) {
        stats->attempts = (int64_t)cs.attempts;
        stats->flips = (int64_t)cs.flips;
        stats->sweeps_max = (int64_t)cs.sweeps_max;
        stats->n_unconverged = (int32_t)cs.unconverged;
        stats->schedule_used = SG_SCHED_FM;
        stats->kernel_ms = ms;
    }
    if (p->until_converged && cs.unconverged)
        return fail(SG_ENOTCONV, "%llu replicas did not converge within %d passes", (unsigned long long)cs.unconverged,
                    p->max_sweeps);
    return SG_OK;
}

}  // namespace

// Error reporting and validation for the library's other translation units.
sg_status sg_internal_fail(sg_status code, const char* msg) { return fail(code, "%s", msg); }

// sg_bind_noalloc's binding: no pinned host buffer is allocated (one from an
// earlier binding is kept).
sg_status bind_impl(sg_handle H, void* dev_ptr, uint64_t bytes, void* hip_stream, bool may_alloc);
sg_status sg_internal_bind(sg_handle H, void* dev_ptr, uint64_t bytes, void* hip_stream, bool may_alloc)
{
    return bind_impl(H, dev_ptr, bytes, hip_stream, may_alloc);
}

sg_status sg_internal_validate(const sg_instance_desc* d) { return validate(*d, 0); }

// ---------------------------------------------------------------------------
// C-ABI

// A drawn start leaves its energy out when the kernel that SG_SCHED_AUTO
// would run next computes the energies of the final spins itself: the
// bit-sliced block kernel for lane-started instances (always), for the
// others the queue kernel (at convergence) or the bit-plane lattice tile
// kernel (taken only when every unit-started instance would run on one of
// these two).  A wrong guess costs an energy pass, never a wrong energy.
bool defer_lane_energy(const sg_ctx* H, const HostInst& q)
{
    return H->defer_energy && H->block_bits && q.bits_ok && !q.lat_ok && q.R >= H->block_min_restarts &&
           can_block(H, q) && bits_lds_for(H, q) > 0;
}

// The lattice schedule would run this instance on the bit-plane tile kernel
// (unless no tiling of it fits, which the run reports through e_written).
bool lattice_msc_bound(const sg_ctx* H, const HostInst& q)
{
    return q.lat_ok && q.lat_msc && H->lattice_msc && !lattice_wg_fits(H, q);
}

bool defer_unit_energy(const sg_ctx* H)
{
    if (!H->defer_energy || H->h_esegs.empty()) return false;
    int64_t queue_items = 0;
    for (const HostInst& q : H->insts)
        if (!q.lat_ok && can_queue(q) && !(q.R >= H->block_min_restarts && can_block(H, q))) queue_items += q.R;
    for (const HostInst& q : H->insts) {
        if (q.dense || (H->lanes_on && lane_start_candidate(q))) continue;
        const bool queue = !q.lat_ok && !(q.R >= H->block_min_restarts && can_block(H, q)) && can_queue(q) &&
                           queue_items >= H->queue_min_items;
        if (!queue && !lattice_msc_bound(H, q)) return false;
    }
    return true;
}

// The run writes the final energies of a deferred instance itself.
bool run_writes_energy(const sg_ctx* H, const sg_run_params* p, int kind, int sched, const HostInst& q)
{
    if (kind == 1) return sched == SG_SCHED_BLOCK && bits_path(H, p, q);
    if (sched == SG_SCHED_LATTICE) return lattice_msc_bound(H, q) && !p->until_converged && p->max_sweeps > 0;
    return sched == SG_SCHED_QUEUE && p->until_converged && p->max_sweeps > 0;
}

// Compute the energies of the current spins of every replica started by the
// unit and lane kernels (those not left out are recomputed unchanged: this
// runs only while no sweep has moved them since their start, or right after
// the run whose final energies it replaces).
sg_status ensure_energy(sg_handle H)
{
    if (!H->e_pending) return SG_OK;
    if (!H->h_eunits.empty())
        SG_HIP(sg::launch_start_units(H->at<sg::InstTab>(H->off_tab), nullptr, 0, H->at<sg::StartUnit>(H->off_eunits),
                                      (int64_t)H->h_eunits.size(), H->at<sg::EnergySeg>(H->off_esegs),
                                      (int64_t)H->h_esegs.size(), H->at<int64_t>(H->off_eparts), H->reps(), nullptr, 0,
                                      false, H->stream),
               "energy kernel");
    if (!H->h_litems.empty())
        SG_HIP(sg::launch_start_lanes(H->at<sg::InstTab>(H->off_tab), H->at<sg::BlockItem>(H->off_litems),
                                      (int)H->h_litems.size(), H->lane_nmax, false, H->reps(), nullptr, 0, H->stream),
               "lane energy kernel");
    H->e_pending = false;
    return SG_OK;
}

extern "C" {

const char* sg_last_error(void) { return g_err.c_str(); }

const char* sg_version(void) { return "sg 0.1 (gfx950)"; }

sg_status sg_load_instance(const sg_instance_desc* descs, int32_t count, sg_handle* out)
{
    g_err.clear();
    if (!descs || !out || count < 1) return fail(SG_EINVAL, "sg_load_instance: need descs, out and count >= 1");
    *out = nullptr;
    sg_ctx* H = new (std::nothrow) sg_ctx;
    if (!H) return fail(SG_ENOMEM, "out of host memory");
    try {
        H->insts.resize((size_t)count);
        for (int32_t k = 0; k < count; ++k) {
            sg_status st = ingest(descs[k], k, H->insts[k]);
            if (st != SG_OK) {
                delete H;
                return st;
            }
            H->insts[k].rep_base = H->total_reps;
            H->total_reps += H->insts[k].R;
        }
        layout(H);
        H->started.assign((size_t)H->total_reps, 0);
    } catch (const std::bad_alloc&) {
        delete H;
        return fail(SG_ENOMEM, "out of host memory while packing instances");
    }
    *out = H;
    return SG_OK;
}

sg_status sg_load_dense(const sg_dense_desc* descs, int32_t count, sg_handle* out)
{
    g_err.clear();
    if (!descs || !out || count < 1) return fail(SG_EINVAL, "sg_load_dense: need descs, out and count >= 1");
    *out = nullptr;
    sg_ctx* H = new (std::nothrow) sg_ctx;
    if (!H) return fail(SG_ENOMEM, "out of host memory");
    try {
        H->dense = 1;
        H->insts.resize((size_t)count);
        for (int32_t k = 0; k < count; ++k) {
            sg_status st = ingest_dense(descs[k], k, H->insts[k]);
            if (st != SG_OK) {
                delete H;
                return st;
            }
            H->insts[k].rep_base = H->total_reps;
            H->total_reps += H->insts[k].R;
        }
        layout(H);
        H->started.assign((size_t)H->total_reps, 0);
    } catch (const std::bad_alloc&) {
        delete H;
        return fail(SG_ENOMEM, "out of host memory while packing instances");
    }
    *out = H;
    return SG_OK;
}

sg_status sg_workspace_bytes(sg_handle H, uint64_t* bytes)
{
    if (!H || !bytes) return fail(SG_EINVAL, "sg_workspace_bytes: null argument");
    *bytes = H->bytes;
    return SG_OK;
}

sg_status sg_instance_info_get(sg_handle H, int32_t inst, sg_instance_info* info, int32_t* colour_out)
{
    if (!H) return fail(SG_EINVAL, "null handle");
    if (inst < 0 || inst >= (int32_t)H->insts.size()) return fail(SG_EINVAL, "instance index %d out of range", inst);
    const HostInst& q = H->insts[inst];
    if (info) {
        info->n = q.n;
        info->colours = q.C;
        info->m = q.m;
        info->t = q.t;
        info->restarts = q.R;
        info->lattice = q.lat_ok;
        info->replica_base = q.rep_base;
    }
    if (colour_out) std::memcpy(colour_out, q.colour.data(), sizeof(int32_t) * (size_t)q.n);
    return SG_OK;
}

}  // extern "C"

sg_status bind_impl(sg_handle H, void* dev_ptr, uint64_t bytes, void* hip_stream, bool may_alloc)
{
    if (!H) return fail(SG_EINVAL, "null handle");
    if (!dev_ptr) return fail(SG_EINVAL, "sg_bind: null device pointer");
    if ((uintptr_t)dev_ptr % kAlign) return fail(SG_EINVAL, "sg_bind: device pointer not 256-byte aligned");
    if (bytes < H->bytes)
        return fail(SG_ENOMEM, "sg_bind: workspace of %llu bytes, need %llu", (unsigned long long)bytes,
                    (unsigned long long)H->bytes);
    H->dev = (uint8_t*)dev_ptr;
    H->stream = (hipStream_t)hip_stream;
    H->bound = false;
    H->stats_zero = false;
    std::fill(H->started.begin(), H->started.end(), 0);
    H->e_pending = false;
    H->e_deferred.assign(H->insts.size(), 0);
    hipStream_t st = H->stream;
    for (const HostInst& q : H->insts) {
        SG_HIP(hipMemcpyAsync(H->dev + q.off_nbr, q.nbr.data(), q.nbr.size() * 4, hipMemcpyHostToDevice, st),
               "upload couplings");
        SG_HIP(hipMemcpyAsync(H->dev + q.off_ta, q.ta.data(), q.ta.size() * 4, hipMemcpyHostToDevice, st),
               "upload triples");
        SG_HIP(hipMemcpyAsync(H->dev + q.off_tb, q.tb.data(), q.tb.size() * 4, hipMemcpyHostToDevice, st),
               "upload triples");
        SG_HIP(hipMemcpyAsync(H->dev + q.off_h, q.h.data(), q.h.size(), hipMemcpyHostToDevice, st), "upload fields");
        if (q.wide) {
            SG_HIP(hipMemcpyAsync(H->dev + q.off_wnbr, q.w_nbr.data(), q.w_nbr.size() * 4, hipMemcpyHostToDevice, st),
                   "upload couplings");
            SG_HIP(hipMemcpyAsync(H->dev + q.off_wJ, q.w_J.data(), q.w_J.size() * 4, hipMemcpyHostToDevice, st),
                   "upload couplings");
            SG_HIP(hipMemcpyAsync(H->dev + q.off_wta, q.w_ta.data(), q.w_ta.size() * 4, hipMemcpyHostToDevice, st),
                   "upload triples");
            SG_HIP(hipMemcpyAsync(H->dev + q.off_wtb, q.w_tb.data(), q.w_tb.size() * 4, hipMemcpyHostToDevice, st),
                   "upload triples");
            SG_HIP(hipMemcpyAsync(H->dev + q.off_wK, q.w_K.data(), q.w_K.size() * 4, hipMemcpyHostToDevice, st),
                   "upload triples");
            SG_HIP(hipMemcpyAsync(H->dev + q.off_wh, q.w_h.data(), q.w_h.size() * 4, hipMemcpyHostToDevice, st),
                   "upload fields");
            SG_HIP(hipMemcpyAsync(H->dev + q.off_wslices, q.w_slices.data(), q.w_slices.size() * sizeof(sg::WSlice),
                                  hipMemcpyHostToDevice, st),
                   "upload slices");
        }
        if (!q.eterm.empty())
            SG_HIP(hipMemcpyAsync(H->dev + q.off_eterm, q.eterm.data(), q.eterm.size() * 4, hipMemcpyHostToDevice, st),
                   "upload energy terms");
        SG_HIP(hipMemcpyAsync(H->dev + q.off_ext, q.ext_of.data(), (size_t)q.n * 4, hipMemcpyHostToDevice, st),
               "upload index map");
        SG_HIP(hipMemcpyAsync(H->dev + q.off_slices, q.slices.data(), q.slices.size() * sizeof(sg::Slice),
                              hipMemcpyHostToDevice, st),
               "upload slices");
        if (q.lat_ok)
            SG_HIP(hipMemcpyAsync(H->dev + q.off_lat_rec, q.lat_rec.data(), q.lat_rec.size() * 8,
                                  hipMemcpyHostToDevice, st),
                   "upload lattice records");
        if (q.dense) {
            SG_HIP(hipMemcpyAsync(H->dev + q.off_dstart, q.d_start.data(), q.d_start.size() * 4, hipMemcpyHostToDevice,
                                  st),
                   "upload terms");
            SG_HIP(hipMemcpyAsync(H->dev + q.off_dmask, q.d_mask.data(), q.d_mask.size() * 8, hipMemcpyHostToDevice, st),
                   "upload terms");
            SG_HIP(hipMemcpyAsync(H->dev + q.off_dcoef, q.d_coef.data(), q.d_coef.size() * 8, hipMemcpyHostToDevice, st),
                   "upload terms");
            SG_HIP(hipMemcpyAsync(H->dev + q.off_tmask, q.t_mask.data(), q.t_mask.size() * 8, hipMemcpyHostToDevice, st),
                   "upload terms");
            SG_HIP(hipMemcpyAsync(H->dev + q.off_tcoef, q.t_coef.data(), q.t_coef.size() * 8, hipMemcpyHostToDevice, st),
                   "upload terms");
            SG_HIP(hipMemcpyAsync(H->dev + q.off_dorder, q.d_order.data(), q.d_order.size() * 4, hipMemcpyHostToDevice,
                                  st),
                   "upload sweep order");
        }
    }
    if (H->dense) {
        std::vector<sg::DenseTab> dt(H->insts.size());
        for (size_t k = 0; k < H->insts.size(); ++k) {
            const HostInst& q = H->insts[k];
            sg::DenseTab& T = dt[k];
            T.dstart = H->at<int32_t>(q.off_dstart);
            T.dmask = H->at<uint64_t>(q.off_dmask);
            T.dcoef = H->at<int64_t>(q.off_dcoef);
            T.tmask = H->at<uint64_t>(q.off_tmask);
            T.tcoef = H->at<int64_t>(q.off_tcoef);
            T.order = H->at<int32_t>(q.off_dorder);
            T.spins = H->at<int8_t>(q.off_spins);
            T.spin_stride = (int64_t)q.spin_stride;
            T.rep_base = q.rep_base;
            T.n = q.n;
            T.nterms = (int32_t)q.t_mask.size();
            T.instance_id = q.id;
            T.pad = 0;
        }
        SG_HIP(hipMemcpyAsync(H->dev + H->off_dtab, dt.data(), dt.size() * sizeof(sg::DenseTab), hipMemcpyHostToDevice,
                              st),
               "upload dense table");
        SG_HIP(hipMemcpyAsync(H->dev + H->off_ditems, H->h_ditems.data(), H->h_ditems.size() * sizeof(sg::BlockItem),
                              hipMemcpyHostToDevice, st),
               "upload dense items");
    }
    std::vector<int64_t> rb(H->insts.size());
    std::vector<int32_t> rr(H->insts.size());
    for (size_t k = 0; k < H->insts.size(); ++k) {
        rb[k] = H->insts[k].rep_base;
        rr[k] = H->insts[k].R;
    }
    SG_HIP(hipMemcpyAsync(H->dev + H->off_rep_base, rb.data(), rb.size() * 8, hipMemcpyHostToDevice, st), "upload");
    SG_HIP(hipMemcpyAsync(H->dev + H->off_restarts, rr.data(), rr.size() * 4, hipMemcpyHostToDevice, st), "upload");
    {
        std::vector<sg::InstTab> tab(H->insts.size());
        std::vector<int32_t> ctab;
        ctab.reserve((size_t)H->ctab_len);
        for (size_t k = 0; k < H->insts.size(); ++k) {
            const HostInst& q = H->insts[k];
            sg::InstTab& T = tab[k];
            T.I = H->view(q);
            T.spins = H->at<int8_t>(q.off_spins);
            T.spin_stride = (int64_t)q.spin_stride;
            T.rep_base = q.rep_base;
            T.C = q.C;
            T.ctab_off = (int32_t)ctab.size();
            T.nbr_words = (int32_t)q.nbr.size();
            T.tri_words = (int32_t)q.ta.size();
            T.eterm = H->at<uint32_t>(q.off_eterm);
            T.n_eh = q.n_eh;
            T.n_ee = q.n_ee;
            T.n_et = q.n_et;
            T.eterm_pad = 0;
            T.fml = q.fml_off == UINT64_MAX ? nullptr : H->at<uint32_t>(H->off_fml) + q.fml_off;
            T.fml_dc = q.fml_dc;
            T.fml_tt = q.fml_tt;
            for (int32_t c = 0; c <= q.C; ++c) ctab.push_back(q.colour_slice[c]);
        }
        SG_HIP(hipMemcpyAsync(H->dev + H->off_tab, tab.data(), tab.size() * sizeof(sg::InstTab), hipMemcpyHostToDevice,
                              st),
               "upload instance table");
        if (!H->h_fml.empty())
            SG_HIP(hipMemcpyAsync(H->dev + H->off_fml, H->h_fml.data(), H->h_fml.size() * 4, hipMemcpyHostToDevice, st),
                   "upload term lists");
        if (H->fmb_nmax > 0) {
            // term rows in external order, their table, the replica items
            std::vector<sg::FmbRows> ptr(H->insts.size(), sg::FmbRows{nullptr, 0, 0, 0, 0});
            std::vector<sg::QueueItem> items;
            std::vector<uint32_t> rows;
            for (size_t k = 0; k < H->insts.size(); ++k) {
                const HostInst& q = H->insts[k];
                if (q.off_fmb_rows == UINT64_MAX) continue;
                build_fmb_rows(q, rows);
                SG_HIP(hipMemcpy(H->dev + q.off_fmb_rows, rows.data(), rows.size() * 4, hipMemcpyHostToDevice),
                       "upload pass rows");
                ptr[k] = sg::FmbRows{H->at<uint32_t>(q.off_fmb_rows), fmb_stride(q), q.fmb_dc, q.fmb_tt, q.wide};
                for (int32_t r = 0; r < q.R; ++r) items.push_back(sg::QueueItem{(int32_t)k, r});
            }
            SG_HIP(hipMemcpy(H->dev + H->off_fmb_ptr, ptr.data(), ptr.size() * sizeof(sg::FmbRows),
                             hipMemcpyHostToDevice),
                   "upload pass row table");
            SG_HIP(hipMemcpy(H->dev + H->off_fmb_items, items.data(), items.size() * sizeof(sg::QueueItem),
                             hipMemcpyHostToDevice),
                   "upload pass items");
        }
        SG_HIP(hipMemcpyAsync(H->dev + H->off_ctab, ctab.data(), ctab.size() * 4, hipMemcpyHostToDevice, st),
               "upload colour table");
        std::vector<int32_t> rep_inst((size_t)H->total_reps);
        for (size_t k = 0; k < H->insts.size(); ++k) {
            const HostInst& q = H->insts[k];
            for (int32_t r = 0; r < q.R; ++r) rep_inst[(size_t)(q.rep_base + r)] = (int32_t)k;
        }
        SG_HIP(hipMemcpyAsync(H->dev + H->off_rep_inst, rep_inst.data(), rep_inst.size() * 4, hipMemcpyHostToDevice,
                              st),
               "upload replica table");
        if (!H->h_sunits.empty())
            SG_HIP(hipMemcpyAsync(H->dev + H->off_sunits, H->h_sunits.data(), H->h_sunits.size() * sizeof(sg::StartUnit),
                                  hipMemcpyHostToDevice, st),
                   "upload start units");
        if (!H->h_eunits.empty()) {
            SG_HIP(hipMemcpyAsync(H->dev + H->off_eunits, H->h_eunits.data(), H->h_eunits.size() * sizeof(sg::StartUnit),
                                  hipMemcpyHostToDevice, st),
                   "upload energy units");
            SG_HIP(hipMemcpyAsync(H->dev + H->off_esegs, H->h_esegs.data(), H->h_esegs.size() * sizeof(sg::EnergySeg),
                                  hipMemcpyHostToDevice, st),
                   "upload energy segments");
        }
        if (!H->h_litems.empty())
            SG_HIP(hipMemcpyAsync(H->dev + H->off_litems, H->h_litems.data(), H->h_litems.size() * sizeof(sg::BlockItem),
                                  hipMemcpyHostToDevice, st),
                   "upload start items");
        SG_HIP(hipStreamSynchronize(st), "stream sync after upload");
    }
    SG_HIP(hipStreamSynchronize(st), "stream sync after upload");
    if (!H->ev0) SG_HIP(hipEventCreate(&H->ev0), "event create");
    if (!H->evh0) SG_HIP(hipEventCreate(&H->evh0), "event create");
    if (!H->evh1) SG_HIP(hipEventCreate(&H->evh1), "event create");
    if (!H->ev1) SG_HIP(hipEventCreate(&H->ev1), "event create");
    if (!H->pin && may_alloc) SG_HIP(hipHostMalloc((void**)&H->pin, kPinBytes, hipHostMallocDefault), "pinned buffer");
    H->bound = true;
    return SG_OK;
}

extern "C" {

sg_status sg_bind(sg_handle H, void* dev_ptr, uint64_t bytes, void* hip_stream)
{
    return bind_impl(H, dev_ptr, bytes, hip_stream, true);
}

sg_status sg_init_spins(sg_handle H, uint64_t seed)
{
    sg_status s = need_bound(H);
    if (s != SG_OK) return s;
    hipStream_t st = H->stream;
    if (H->dense) {
        SG_HIP(sg::launch_dense_init(H->at<sg::DenseTab>(H->off_dtab), H->at<sg::BlockItem>(H->off_ditems),
                                     (int)H->h_ditems.size(), H->reps(), seed, st),
               "dense init kernel");
        SG_HIP(hipStreamSynchronize(st), "stream sync");
        std::fill(H->started.begin(), H->started.end(), 1);
        return SG_OK;
    }
    H->e_pending = false;
    H->e_deferred.assign(H->insts.size(), 0);
    const bool defer_units = defer_unit_energy(H);
    if (defer_units) {
        for (size_t k = 0; k < H->insts.size(); ++k) {
            const HostInst& q = H->insts[k];
            if (!q.dense && !(H->lanes_on && lane_start_candidate(q))) H->e_deferred[k] = 2;
        }
        H->e_pending = true;
    }
    if (!H->h_sunits.empty())
        SG_HIP(sg::launch_start_units(H->at<sg::InstTab>(H->off_tab), H->at<sg::StartUnit>(H->off_sunits),
                                      (int64_t)H->h_sunits.size(), H->at<sg::StartUnit>(H->off_eunits),
                                      defer_units ? 0 : (int64_t)H->h_eunits.size(),
                                      H->at<sg::EnergySeg>(H->off_esegs), defer_units ? 0 : (int64_t)H->h_esegs.size(),
                                      H->at<int64_t>(H->off_eparts), H->reps(), nullptr, seed, true, st),
               "start kernels");
    if (!H->h_litems.empty()) {
        bool changed = false;
        for (sg::BlockItem& it : H->h_litems) {
            const int32_t d = defer_lane_energy(H, H->insts[(size_t)it.inst]) ? 1 : 0;
            H->e_deferred[(size_t)it.inst] = (uint8_t)d;
            H->e_pending = H->e_pending || d;
            changed = changed || it.pad != d;
            it.pad = d;
        }
        if (changed)
            SG_HIP(hipMemcpyAsync(H->dev + H->off_litems, H->h_litems.data(), H->h_litems.size() * sizeof(sg::BlockItem),
                                  hipMemcpyHostToDevice, st),
                   "upload lane items");
        SG_HIP(sg::launch_start_lanes(H->at<sg::InstTab>(H->off_tab), H->at<sg::BlockItem>(H->off_litems),
                                      (int)H->h_litems.size(), H->lane_nmax, true, H->reps(), nullptr, seed, st),
               "lane start kernel");
    }
    // start energies of the wide-form instances (their starts came from the unit kernel above)
    for (const HostInst& q : H->insts)
        if (q.wide)
            SG_HIP(sg::launch_wide_energy(H->wview(q), H->at<int8_t>(q.off_spins), (int64_t)q.spin_stride, q.R,
                                          H->at<int64_t>(H->off_slots), q.nslots, H->reps() + q.rep_base, nullptr, st),
                   "wide energy kernel");
    // enqueued on the bound stream: every later call of the handle is ordered after it
    std::fill(H->started.begin(), H->started.end(), 1);
    return SG_OK;
}

sg_status sg_set_spins(sg_handle H, int32_t inst, int32_t r, const int8_t* s)
{
    sg_status e = need_bound(H);
    if (e != SG_OK) return e;
    if ((e = check_inst(H, inst, r)) != SG_OK) return e;
    if (!s) return fail(SG_EINVAL, "sg_set_spins: null spins");
    const HostInst& q = H->insts[inst];
    std::vector<int8_t> tmp((size_t)q.n);
    for (int32_t i = 0; i < q.n; ++i) {
        const int8_t v = s[q.ext_of[i]];
        if (v != 1 && v != -1) return fail(SG_EINVAL, "sg_set_spins: spin %u is %d, not +1 or -1", q.ext_of[i], v);
        tmp[i] = v;
    }
    hipStream_t st = H->stream;
    int8_t* dst = H->at<int8_t>(q.off_spins) + (uint64_t)r * q.spin_stride;
    sg::RepState z{};
    sg::RepState* rs = H->reps() + q.rep_base + r;
    if (q.dense) {  // exact energy of the start on the host: E = -sum coef prod s
        for (size_t t = 0; t < q.t_mask.size(); ++t) {
            int64_t prod = 1;
            for (int i = 0; i < q.n; ++i)
                if ((q.t_mask[t] >> i) & 1ull) prod *= tmp[i];
            z.E -= q.t_coef[t] * prod;
        }
    }
    SG_HIP(hipMemcpyAsync(dst, tmp.data(), (size_t)q.n, hipMemcpyHostToDevice, st), "spin upload");
    SG_HIP(hipMemcpyAsync(rs, &z, sizeof z, hipMemcpyHostToDevice, st), "state upload");
    if (q.wide)
        SG_HIP(sg::launch_wide_energy(H->wview(q), dst, (int64_t)q.spin_stride, 1, H->at<int64_t>(H->off_slots),
                                      q.nslots, rs, nullptr, st),
               "wide energy kernel");
    else if (!q.dense)
        SG_HIP(sg::launch_energy(H->view(q), dst, (int64_t)q.spin_stride, 1, H->at<int64_t>(H->off_slots), q.nslots,
                                 rs, nullptr, st),
               "energy kernel");
    SG_HIP(hipStreamSynchronize(st), "stream sync");
    H->started[(size_t)(q.rep_base + r)] = 1;
    return SG_OK;
}

sg_status sg_run_sweeps(sg_handle H, const sg_run_params* p, sg_run_stats* stats)
{
    sg_status e = need_bound(H);
    if (e != SG_OK) return e;
    if (!p) return fail(SG_EINVAL, "sg_run_sweeps: null params");
    if (p->rule != SG_RULE_GREEDY && p->rule != SG_RULE_GREEDY_TIE && p->rule != SG_RULE_FM)
        return fail(SG_EINVAL, "unknown rule %d", p->rule);
    if (p->max_sweeps < 0) return fail(SG_EINVAL, "max_sweeps must be >= 0");
    for (uint8_t v : H->started)
        if (!v) return fail(SG_ESTATE, "a replica has no start (call sg_init_spins or sg_set_spins)");
    H->stats_zero = false;  // every run below leaves its totals there
    if (H->dense) return run_dense(H, p, stats);
    if (p->rule == SG_RULE_FM) {
        if ((e = ensure_energy(H)) != SG_OK) return e;
        return run_fm(H, p, stats);
    }
    std::vector<int> assign;
    const int sched = assign_schedules(H, p, assign);
    if (sched < 0 && p->schedule != SG_SCHED_AUTO)
        return fail(SG_EINVAL, "schedule %d is not available for this handle (rule %d, until_converged %d)",
                    p->schedule, p->rule, p->until_converged);
    // left-out start energies are written by the bit-sliced or the queue
    // kernel; any other kernel continues from them, so they are computed first
    for (size_t k = 0; H->e_pending && k < assign.size(); ++k)
        if (H->e_deferred[k] && !run_writes_energy(H, p, H->e_deferred[k], assign[k], H->insts[k]))
            if ((e = ensure_energy(H)) != SG_OK) return e;
    hipStream_t st = H->stream;
    SG_HIP(sg::launch_fill_u32(H->at<uint32_t>(H->off_stats), sizeof(sg::CallStats) / 4, 0u, st), "fill kernel");
    SG_HIP(hipEventRecord(H->ev0, st), "event record");
    H->hot_launches = 0;
    H->lat_err_check = false;
    H->e_written.assign(H->insts.size(), 0);
    for (int kind : {SG_SCHED_LATTICE, SG_SCHED_BLOCK, SG_SCHED_QUEUE, SG_SCHED_GRAPH, SG_SCHED_FIELDS, SG_SCHED_PHASE}) {
        std::vector<int> which;
        for (size_t k = 0; k < assign.size(); ++k)
            if (assign[k] == kind) which.push_back((int)k);
        if (which.empty()) continue;
        switch (kind) {
        case SG_SCHED_LATTICE: e = run_lattice_schedule(H, p, which); break;
        case SG_SCHED_BLOCK: e = run_block_schedule(H, p, which); break;
        case SG_SCHED_QUEUE: e = run_queue_schedule(H, p, which); break;
        case SG_SCHED_GRAPH: e = run_graph_schedule(H, p, which); break;
        case SG_SCHED_FIELDS: e = run_phase_schedule(H, p, which, true); break;
        default: e = run_phase_schedule(H, p, which); break;
        }
        if (e != SG_OK) return e;
    }
    SG_HIP(hipEventRecord(H->ev1, st), "event record");
    sg::CallStats cs;
    uint32_t herr = 0;
    CopiesOut out(H);
    SG_HIP(out.copy(&cs, H->at<sg::CallStats>(H->off_stats), sizeof cs, st), "stats copy");
    if (H->lat_err_check) SG_HIP(out.copy(&herr, H->at<uint32_t>(H->off_err), 4, st), "error flag copy");
    SG_HIP(hipStreamSynchronize(st), "stream sync");
    out.finish();
    if (herr)
        return fail(SG_EDEVICE, "lattice tile kernel: a neighbour wait timed out (replica state is undefined; "
                                "start again with sg_init_spins)");
    if (H->e_pending) {
        // the queue kernel wrote the energies of the replicas that converged,
        // the bit-plane lattice kernel those of its instances; if any replica
        // is left without, all are computed from their final spins
        bool missing = false;
        for (size_t k = 0; k < H->e_deferred.size(); ++k) {
            if (H->e_deferred[k] != 2) continue;
            if (assign[k] == SG_SCHED_QUEUE) missing = missing || cs.unconverged != 0;
            else missing = missing || !H->e_written[k];
        }
        if (missing) {
            if ((e = ensure_energy(H)) != SG_OK) return e;
            SG_HIP(hipStreamSynchronize(st), "stream sync");
        }
        H->e_pending = false;
    }
    float ms = 0.f;
    SG_HIP(hipEventElapsedTime(&ms, H->ev0, H->ev1), "event time");
    H->hot_us = 0.0;
    if (H->hot_launches > 0) {
        float hms = 0.f;
        if (hipEventElapsedTime(&hms, H->evh0, H->evh1) == hipSuccess) H->hot_us = hms * 1000.0;
        else (void)hipGetLastError();
    }
    if (stats) {
        stats->attempts = (int64_t)cs.attempts;
        stats->flips = (int64_t)cs.flips;
        stats->sweeps_max = (int64_t)cs.sweeps_max;
        stats->n_unconverged = (int32_t)cs.unconverged;
        stats->schedule_used = sched;
        stats->kernel_ms = ms;
    }
    if (p->until_converged && cs.unconverged) {
        fail(SG_ENOTCONV, "%llu replicas did not converge within %d sweeps", (unsigned long long)cs.unconverged,
             p->max_sweeps);
        return SG_ENOTCONV;
    }
    return SG_OK;
}

sg_status sg_energy(sg_handle H, int64_t* E, int32_t recompute)
{
    sg_status e = need_bound(H);
    if (e != SG_OK) return e;
    if (!E) return fail(SG_EINVAL, "sg_energy: null output");
    if (!recompute && (e = ensure_energy(H)) != SG_OK) return e;
    hipStream_t st = H->stream;
    if (recompute) {
        int64_t* eout = H->at<int64_t>(H->off_eout);
        if (H->dense)
            SG_HIP(sg::launch_dense_energy(H->at<sg::DenseTab>(H->off_dtab), H->at<sg::BlockItem>(H->off_ditems),
                                           (int)H->h_ditems.size(), eout, st),
                   "dense energy kernel");
        if (!H->h_eunits.empty()) {
            SG_HIP(sg::launch_fill_u32(reinterpret_cast<uint32_t*>(eout), (uint64_t)H->total_reps * 2, 0u, st),
                   "fill kernel");
            SG_HIP(sg::launch_start_units(H->at<sg::InstTab>(H->off_tab), nullptr, 0, H->at<sg::StartUnit>(H->off_eunits),
                                          (int64_t)H->h_eunits.size(), H->at<sg::EnergySeg>(H->off_esegs),
                                          (int64_t)H->h_esegs.size(), H->at<int64_t>(H->off_eparts), H->reps(), eout,
                                          0, false, st),
                   "energy kernel");
        }
        if (!H->h_litems.empty())
            SG_HIP(sg::launch_start_lanes(H->at<sg::InstTab>(H->off_tab), H->at<sg::BlockItem>(H->off_litems),
                                          (int)H->h_litems.size(), H->lane_nmax, false, H->reps(), eout, 0, st),
                   "batched energy kernel");
        for (const HostInst& q : H->insts)
            if (q.wide)
                SG_HIP(sg::launch_wide_energy(H->wview(q), H->at<int8_t>(q.off_spins), (int64_t)q.spin_stride, q.R,
                                              H->at<int64_t>(H->off_slots), q.nslots, nullptr, eout + q.rep_base, st),
                       "wide energy kernel");
        SG_HIP(hipMemcpyAsync(E, eout, (size_t)H->total_reps * 8, hipMemcpyDeviceToHost, st), "energy copy");
        SG_HIP(hipStreamSynchronize(st), "stream sync");
        return SG_OK;
    }
    std::vector<sg::RepState> rs((size_t)H->total_reps);
    CopiesOut out(H);
    SG_HIP(out.copy(rs.data(), H->reps(), rs.size() * sizeof(sg::RepState), st), "state copy");
    SG_HIP(hipStreamSynchronize(st), "stream sync");
    out.finish();
    for (size_t k = 0; k < rs.size(); ++k) E[k] = rs[k].E;
    return SG_OK;
}

sg_status sg_replica_counters(sg_handle H, int64_t* sweeps, int64_t* flips, int8_t* converged)
{
    sg_status e = need_bound(H);
    if (e != SG_OK) return e;
    std::vector<sg::RepState> rs((size_t)H->total_reps);
    SG_HIP(hipMemcpyAsync(rs.data(), H->reps(), rs.size() * sizeof(sg::RepState), hipMemcpyDeviceToHost, H->stream),
           "state copy");
    SG_HIP(hipStreamSynchronize(H->stream), "stream sync");
    for (size_t k = 0; k < rs.size(); ++k) {
        if (sweeps) sweeps[k] = rs[k].sweeps;
        if (flips) flips[k] = rs[k].flips;
        if (converged) converged[k] = (int8_t)rs[k].converged;
    }
    return SG_OK;
}

sg_status sg_spins_out(sg_handle H, int32_t inst, int32_t r, int8_t* s)
{
    sg_status e = need_bound(H);
    if (e != SG_OK) return e;
    if ((e = check_inst(H, inst, r)) != SG_OK) return e;
    if (!s) return fail(SG_EINVAL, "sg_spins_out: null output");
    const HostInst& q = H->insts[inst];
    std::vector<int8_t> tmp((size_t)q.n);
    SG_HIP(hipMemcpyAsync(tmp.data(), H->at<int8_t>(q.off_spins) + (uint64_t)r * q.spin_stride, (size_t)q.n,
                          hipMemcpyDeviceToHost, H->stream),
           "spin copy");
    SG_HIP(hipStreamSynchronize(H->stream), "stream sync");
    for (int32_t i = 0; i < q.n; ++i) s[q.ext_of[i]] = tmp[i];
    return SG_OK;
}

sg_status sg_spins_out_batch(sg_handle H, int32_t inst, int32_t r0, int32_t count, int8_t* s)
{
    sg_status e = need_bound(H);
    if (e != SG_OK) return e;
    if (count < 1 || !s) return fail(SG_EINVAL, "sg_spins_out_batch: need count >= 1 and an output");
    if ((e = check_inst(H, inst, r0)) != SG_OK) return e;
    if ((e = check_inst(H, inst, r0 + count - 1)) != SG_OK) return e;
    const HostInst& q = H->insts[inst];
    std::vector<int8_t> tmp((size_t)q.spin_stride * count);
    SG_HIP(hipMemcpyAsync(tmp.data(), H->at<int8_t>(q.off_spins) + (uint64_t)r0 * q.spin_stride, tmp.size(),
                          hipMemcpyDeviceToHost, H->stream),
           "spin copy");
    SG_HIP(hipStreamSynchronize(H->stream), "stream sync");
    for (int32_t r = 0; r < count; ++r) {
        const int8_t* src = tmp.data() + (size_t)r * q.spin_stride;
        int8_t* dst = s + (size_t)r * q.n;
        for (int32_t i = 0; i < q.n; ++i) dst[q.ext_of[i]] = src[i];
    }
    return SG_OK;
}

sg_status sg_best(sg_handle H, int64_t* E_best, int32_t* r_best)
{
    sg_status e = need_bound(H);
    if (e != SG_OK) return e;
    if ((e = ensure_energy(H)) != SG_OK) return e;
    const int ni = (int)H->insts.size();
    hipStream_t st = H->stream;
    SG_HIP(sg::launch_best(H->reps(), H->at<int64_t>(H->off_rep_base), H->at<int32_t>(H->off_restarts), ni,
                           H->at<int64_t>(H->off_best_E), H->at<int32_t>(H->off_best_r), st),
           "best kernel");
    std::vector<int64_t> eb((size_t)ni);
    std::vector<int32_t> rb((size_t)ni);
    CopiesOut out(H);
    SG_HIP(out.copy(eb.data(), H->at<int64_t>(H->off_best_E), (size_t)ni * 8, st), "copy");
    SG_HIP(out.copy(rb.data(), H->at<int32_t>(H->off_best_r), (size_t)ni * 4, st), "copy");
    SG_HIP(hipStreamSynchronize(st), "stream sync");
    out.finish();
    if (E_best) std::memcpy(E_best, eb.data(), (size_t)ni * 8);
    if (r_best) std::memcpy(r_best, rb.data(), (size_t)ni * 4);
    return SG_OK;
}

sg_status sg_solve(sg_handle H, const sg_run_params* p, sg_run_stats* stats, int64_t* E_best, int32_t* r_best)
{
    sg_status e = need_bound(H);
    if (e != SG_OK) return e;
    if (!p) return fail(SG_EINVAL, "sg_solve: null params");
    if (p->rule != SG_RULE_GREEDY && p->rule != SG_RULE_GREEDY_TIE && p->rule != SG_RULE_FM)
        return fail(SG_EINVAL, "unknown rule %d", p->rule);
    if (p->max_sweeps < 0) return fail(SG_EINVAL, "max_sweeps must be >= 0");
    // one launch per instance when every instance is a lattice that the
    // workgroup-per-replica kernel holds and the run would take that kernel
    bool one = !H->dense && (p->rule == SG_RULE_GREEDY || p->rule == SG_RULE_GREEDY_TIE) && p->max_sweeps >= 0 &&
               (p->schedule == SG_SCHED_AUTO || p->schedule == SG_SCHED_LATTICE) && !H->insts.empty();
    for (const HostInst& q : H->insts) one = one && !q.wide && q.lat_ok && lattice_wg_fits(H, q);
    if (one) {
        std::vector<int> assign;
        one = assign_schedules(H, p, assign) == SG_SCHED_LATTICE;
    }
    if (!one) {
        if ((e = sg_init_spins(H, p->seed)) != SG_OK) return e;
        const sg_status run = sg_run_sweeps(H, p, stats);
        if (run < 0) return run;
        if ((e = sg_best(H, E_best, r_best)) != SG_OK) return e;
        return run;
    }
    hipStream_t st = H->stream;
    const int ni = (int)H->insts.size();
    sg::CallStats* cs = H->at<sg::CallStats>(H->off_stats);
    // results of the call, written by the last workgroup of each launch: call
    // totals (64 bytes), best energies, best restarts; read back in one copy
    static_assert(sizeof(sg::CallStats) <= 64, "the call totals take the first 64 bytes of the results");
    uint8_t* res = H->dev + H->off_solve;
    const size_t res_bytes = 64 + (size_t)ni * 12;
    if (!H->stats_zero)
        SG_HIP(sg::launch_fill_u32(H->at<uint32_t>(H->off_stats), sizeof(sg::CallStats) / 4, 0u, st), "fill kernel");
    H->stats_zero = false;
    SG_HIP(hipEventRecord(H->ev0, st), "event record");
    unsigned long long done_end = 0;
    for (int k = 0; k < ni; ++k) {
        const HostInst& q = H->insts[(size_t)k];
        done_end += (unsigned long long)q.R;
        const sg::WgSolve sv{cs, reinterpret_cast<int64_t*>(res + 64) + k,
                             reinterpret_cast<int32_t*>(res + 64 + (size_t)ni * 8) + k,
                             k == ni - 1 ? reinterpret_cast<sg::CallStats*>(res) : nullptr, done_end};
        SG_HIP(sg::launch_lattice_wg(H->lat_view(q), H->at<int8_t>(q.off_spins), (int64_t)q.spin_stride,
                                     H->reps() + q.rep_base, q.R, nullptr, 0, p->max_sweeps, p->seed, p->rule,
                                     p->until_converged, st, &sv),
               "lattice workgroup kernel");
    }
    SG_HIP(hipEventRecord(H->ev1, st), "event record");
    H->hot_launches = ni;
    std::vector<uint8_t> hres(res_bytes);
    CopiesOut out(H);
    SG_HIP(out.copy(hres.data(), res, res_bytes, st), "result copy");
    SG_HIP(hipStreamSynchronize(st), "stream sync");
    out.finish();
    H->stats_zero = true;
    sg::CallStats c;
    std::memcpy(&c, hres.data(), sizeof c);
    std::vector<int64_t> eb((size_t)ni);
    std::vector<int32_t> rb((size_t)ni);
    std::memcpy(eb.data(), hres.data() + 64, (size_t)ni * 8);
    std::memcpy(rb.data(), hres.data() + 64 + (size_t)ni * 8, (size_t)ni * 4);
    // every replica has a start and an exact energy
    std::fill(H->started.begin(), H->started.end(), 1);
    H->e_pending = false;
    H->e_deferred.assign(H->insts.size(), 0);
    float ms = 0.f;
    SG_HIP(hipEventElapsedTime(&ms, H->ev0, H->ev1), "event time");
    H->hot_us = ms * 1000.0;  // only the solve's launches lie between the events
    if (E_best) std::memcpy(E_best, eb.data(), (size_t)ni * 8);
    if (r_best) std::memcpy(r_best, rb.data(), (size_t)ni * 4);
    if (stats) {
        stats->attempts = (int64_t)c.attempts;
        stats->flips = (int64_t)c.flips;
        stats->sweeps_max = (int64_t)c.sweeps_max;
        stats->n_unconverged = (int32_t)c.unconverged;
        stats->schedule_used = SG_SCHED_LATTICE;
        stats->kernel_ms = ms;
    }
    if (p->until_converged && c.unconverged) {
        fail(SG_ENOTCONV, "%llu replicas did not converge within %d sweeps", (unsigned long long)c.unconverged,
             p->max_sweeps);
        return SG_ENOTCONV;
    }
    return SG_OK;
}

sg_status sg_tune(sg_handle H, const char* key, int64_t value)
{
    if (!H || !key) return fail(SG_EINVAL, "sg_tune: null argument");
    const std::string k(key);
    if (k == "lattice_k") {
        if (value < 1 || value > 16) return fail(SG_EINVAL, "lattice_k must be in [1,16]");
        H->lattice_k = (int32_t)value;
    } else if (k == "lattice_max_tiles") {
        if (value < 0 || value > kMaxLatticeTiles) return fail(SG_EINVAL, "lattice_max_tiles out of range");
        H->lattice_max_tiles = (int32_t)value;
    } else if (k == "lattice_wg_max_n") {
        if (value < 0 || value > 150000) return fail(SG_EINVAL, "lattice_wg_max_n must be in [0,150000]");
        H->lattice_wg_max_n = (int32_t)value;
    } else if (k == "fm_waves") {
        if (value < 0 || value > 16) return fail(SG_EINVAL, "fm_waves must be in [0,16]");
        H->fm_waves = (int32_t)value;
    } else if (k == "fm_key32") {
        if (value != 0 && value != 1) return fail(SG_EINVAL, "fm_key32 must be 0 or 1");
        H->fm_key32 = (int32_t)value;
    } else if (k == "fm_lanes") {
        if (value != 0 && value != 1) return fail(SG_EINVAL, "fm_lanes must be 0 or 1");
        if (!H->bound) {
            // before sg_bind the term lists follow the knob (0 leaves them out of the workspace)
            H->fml_ws = (int32_t)value;
            layout(H);
        } else if (value && !H->fml_ws) {
            return fail(SG_EINVAL, "fm_lanes: the workspace was laid out without the term lists (set it before sg_bind)");
        }
        H->fm_lanes = (int32_t)value;
    } else if (k == "fm_slots") {
        if (value < 0 || value > 65536) return fail(SG_EINVAL, "fm_slots must be in [0,65536]");
        if (H->bound) return fail(SG_EINVAL, "fm_slots sizes the workspace: set it before sg_bind");
        H->fm_slots = (int32_t)value;
        layout(H);
    } else if (k == "fm_lane_waves") {
        if (value < 0 || value > 4) return fail(SG_EINVAL, "fm_lane_waves must be in [0,4]");
        H->fm_lane_waves = (int32_t)value;
    } else if (k == "fm_lane_restarts") {
        if (value < 0 || value > (1 << 20) || value % 64)
            return fail(SG_EINVAL, "fm_lane_restarts must be 0 or a multiple of 64 up to 2^20");
        H->fm_lane_restarts = (int32_t)value;
    } else if (k == "defer_energy") {
        if (value != 0 && value != 1) return fail(SG_EINVAL, "defer_energy must be 0 or 1");
        H->defer_energy = (int32_t)value;
    } else if (k == "block_bits") {
        if (value != 0 && value != 1) return fail(SG_EINVAL, "block_bits must be 0 or 1");
        H->block_bits = (int32_t)value;
    } else if (k == "bits_groups") {
        if (value != 2 && value != 4 && value != 8 && value != 16)
            return fail(SG_EINVAL, "bits_groups must be 2, 4, 8 or 16");
        H->bits_groups = (int32_t)value;
    } else if (k == "block_groups") {
        if (value < 0 || value > 64) return fail(SG_EINVAL, "block_groups must be in [0, 64]");
        H->block_groups = (int32_t)value;
    } else if (k == "block_rg") {
        if (value != 0 && value != 64 && value != 128 && value != 256)
            return fail(SG_EINVAL, "block_rg must be 0, 64, 128 or 256");
        H->block_rg = (int32_t)value;
    } else if (k == "block_min_restarts") {
        if (value < 1) return fail(SG_EINVAL, "block_min_restarts must be >= 1");
        H->block_min_restarts = (int32_t)std::min<int64_t>(value, INT32_MAX);
    } else if (k == "queue_wave_max_n") {
        if (value < 0 || value > 9000) return fail(SG_EINVAL, "queue_wave_max_n must be in [0,9000]");
        H->queue_wave_max_n = (int32_t)value;
    } else if (k == "queue_grid") {
        if (value < 0 || value > 65535) return fail(SG_EINVAL, "queue_grid must be in [0,65535]");
        H->queue_grid = (int32_t)value;
    } else if (k == "lattice_msc") {
        if (value != 0 && value != 1) return fail(SG_EINVAL, "lattice_msc must be 0 or 1");
        H->lattice_msc = (int32_t)value;
    } else if (k == "msc_k") {
        if (value < 0 || value > 62) return fail(SG_EINVAL, "msc_k must be in [0,62]");
        H->msc_k = (int32_t)value;
    } else if (k == "fields") {
        if (value != 0 && value != 1) return fail(SG_EINVAL, "fields must be 0 or 1");
        if (H->bound) return fail(SG_EINVAL, "fields changes the workspace: set it before sg_bind");
        H->fields_ws = (int32_t)value;
        layout(H);
    } else if (k == "graph_sweeps") {
        if (value < 1 || value > 1024) return fail(SG_EINVAL, "graph_sweeps must be in [1,1024]");
        H->graph_sweeps = (int32_t)value;
    } else if (k == "lattice_conv_chunk") {
        if (value < 1 || value > kConvChunk) return fail(SG_EINVAL, "lattice_conv_chunk must be in [1,%d]", kConvChunk);
        H->conv_chunk = (int32_t)value;
    } else if (k == "auto_graph") {
        if (value != 0 && value != 1) return fail(SG_EINVAL, "auto_graph must be 0 or 1");
        H->auto_graph = (int32_t)value;
    } else if (k == "queue_min_items") {
        if (value < 1) return fail(SG_EINVAL, "queue_min_items must be >= 1");
        H->queue_min_items = (int32_t)std::min<int64_t>(value, INT32_MAX);
    } else {
        return fail(SG_EINVAL, "sg_tune: unknown key '%s'", key);
    }
    return SG_OK;
}

sg_status sg_query(sg_handle H, const char* key, int64_t* value)
{
    if (!H || !key || !value) return fail(SG_EINVAL, "sg_query: null argument");
    const std::string k(key);
    if (k == "lattice_k") *value = H->lattice_k;
    else if (k == "lattice_max_tiles") *value = H->lattice_max_tiles;
    else if (k == "lattice_wg_max_n") *value = H->lattice_wg_max_n;
    else if (k == "block_rg") *value = H->block_rg;
    else if (k == "block_groups") *value = H->block_groups;
    else if (k == "block_bits") *value = H->block_bits;
    else if (k == "fm_waves") *value = H->fm_waves;
    else if (k == "last_fm_waves") *value = H->last_fm_waves;
    else if (k == "defer_energy") *value = H->defer_energy;
    else if (k == "energy_pending") *value = H->e_pending ? 1 : 0;
    else if (k == "fm_key32") *value = H->fm_key32;
    else if (k == "fm_lanes") *value = H->fm_lanes;
    else if (k == "fm_lane_restarts") *value = H->fm_lane_restarts;
    else if (k == "fm_lane_waves") *value = H->fm_lane_waves;
    else if (k == "fm_slots") *value = H->fm_slots;
    else if (k == "last_fm_big") *value = H->last_fm_big;
    else if (k == "last_fm_lanes") *value = H->last_fm_lanes;
    else if (k == "last_fm_lane_nr") *value = H->last_fm_lane_nr;
    else if (k == "last_key32") *value = H->last_key32;
    else if (k == "bits_groups") *value = H->bits_groups;
    else if (k == "block_min_restarts") *value = H->block_min_restarts;
    else if (k == "queue_wave_max_n") *value = H->queue_wave_max_n;
    else if (k == "queue_grid") *value = H->queue_grid;
    else if (k == "queue_min_items") *value = H->queue_min_items;
    else if (k == "graph_sweeps") *value = H->graph_sweeps;
    else if (k == "auto_graph") *value = H->auto_graph;
    else if (k == "lattice_conv_chunk") *value = H->conv_chunk;
    else if (k == "fields") *value = H->fields_ws;
    else if (k == "lattice_msc") *value = H->lattice_msc;
    else if (k == "msc_k") *value = H->msc_k;
    else if (k == "last_msc") *value = H->last_msc;
    else if (k == "last_bits") *value = H->last_bits;
    else if (k == "last_queue_grid") *value = H->last_queue_grid;
    else if (k == "hot_ns") *value = (int64_t)(H->hot_us * 1000.0);
    else if (k == "hot_launches") *value = H->hot_launches;
    else if (k == "last_tiles") *value = (int64_t)H->last_tiles[0] * 1000000 + H->last_tiles[1] * 1000 + H->last_tiles[2];
    else if (k == "last_tile_k") *value = H->last_tiles[3];
    else if (k == "last_model_phase_ns") *value = (int64_t)std::llround(H->last_model_phase_us * 1000.0);
    else if (k == "last_model_exchange_ns") *value = (int64_t)std::llround(H->last_model_ex_us * 1000.0);
    else if (k == "last_model_phases") *value = H->last_model_phases;
    else if (k == "last_model_exchanges") *value = H->last_model_exchanges;
    else if (k == "total_replicas") *value = H->total_reps;
    else if (k == "queue_ok") {
        int64_t ok = H->dense ? 0 : 1;
        for (const HostInst& q : H->insts) ok = ok && can_queue(q);
        *value = ok;
    }
    else if (k == "wide_instances") {
        int64_t c = 0;
        for (const HostInst& q : H->insts) c += q.wide;
        *value = c;
    }
    else if (k == "instances") *value = (int64_t)H->insts.size();
    else return fail(SG_EINVAL, "sg_query: unknown key '%s'", key);
    return SG_OK;
}

// ---------------------------------------------------------------------------
// continuous batching: the replicas of several handles in one launch of the
// persistent queue kernel

namespace {

struct GroupLayout {
    uint64_t off_tab = 0, off_ctab = 0, off_items = 0, off_cnt = 0, off_stats = 0, bytes = 0;
    int64_t ninst = 0, nctab = 0, nitems = 0;
};

sg_status group_layout(const sg_handle* hs, int32_t count, GroupLayout& g)
{
    if (!hs || count < 1) return fail(SG_EINVAL, "sg_run_group: need handles and count >= 1");
    for (int32_t k = 0; k < count; ++k) {
        const sg_ctx* H = hs[k];
        if (!H) return fail(SG_EINVAL, "sg_run_group: handle %d is null", k);
        if (H->dense) return fail(SG_EINVAL, "sg_run_group: handle %d holds dense instances", k);
        for (size_t q = 0; q < H->insts.size(); ++q)
            if (!can_queue(H->insts[q]))
                return fail(SG_EINVAL, "sg_run_group: instance %zu of handle %d cannot run on the queue kernel "
                                       "(more than %d spins, or the wide form)", q, k, kQueueMaxN);
        g.ninst += (int64_t)H->insts.size();
        g.nitems += H->total_reps;
        for (const HostInst& q : H->insts) g.nctab += q.C + 1;
    }
    if (g.nitems > INT32_MAX || g.ninst > INT32_MAX || g.nctab > INT32_MAX)
        return fail(SG_ERANGE, "sg_run_group: more than 2^31 - 1 replicas");
    uint64_t off = 0;
    auto take = [&](uint64_t b) {
        const uint64_t o = off;
        off = align_up(off + std::max<uint64_t>(b, 1));
        return o;
    };
    g.off_tab = take((uint64_t)g.ninst * sizeof(sg::InstTab));
    g.off_ctab = take((uint64_t)g.nctab * 4);
    g.off_items = take((uint64_t)g.nitems * sizeof(sg::QueueItem));
    g.off_cnt = take(64);
    g.off_stats = take(sizeof(sg::CallStats));
    g.bytes = off;
    return SG_OK;
}

}  // namespace

sg_status sg_group_scratch_bytes(const sg_handle* hs, int32_t count, uint64_t* bytes)
{
    if (!bytes) return fail(SG_EINVAL, "sg_group_scratch_bytes: null output");
    GroupLayout g;
    sg_status e = group_layout(hs, count, g);
    if (e != SG_OK) return e;
    *bytes = g.bytes;
    return SG_OK;
}

sg_status sg_run_group(const sg_handle* hs, int32_t count, const sg_run_params* p, void* dev_scratch,
                       uint64_t scratch_bytes, int32_t* unconverged, sg_run_stats* stats)
{
    GroupLayout g;
    sg_status e = group_layout(hs, count, g);
    if (e != SG_OK) return e;
    if (!p) return fail(SG_EINVAL, "sg_run_group: null params");
    if (p->rule != SG_RULE_GREEDY && p->rule != SG_RULE_GREEDY_TIE)
        return fail(SG_EINVAL, "sg_run_group: rule %d (the queue kernel runs GREEDY and GREEDY_TIE)", p->rule);
    if (p->schedule != SG_SCHED_AUTO && p->schedule != SG_SCHED_QUEUE)
        return fail(SG_EINVAL, "sg_run_group: schedule %d (a group runs on SG_SCHED_QUEUE)", p->schedule);
    if (p->max_sweeps < 0) return fail(SG_EINVAL, "max_sweeps must be >= 0");
    if (!dev_scratch || ((uintptr_t)dev_scratch % kAlign))
        return fail(SG_EINVAL, "sg_run_group: scratch must be a 256-byte aligned device pointer");
    if (scratch_bytes < g.bytes)
        return fail(SG_ENOMEM, "sg_run_group: scratch of %llu bytes, need %llu", (unsigned long long)scratch_bytes,
                    (unsigned long long)g.bytes);
    sg_ctx* H0 = hs[0];
    for (int32_t k = 0; k < count; ++k) {
        sg_ctx* H = hs[k];
        if ((e = need_bound(H)) != SG_OK) return e;
        if (H->stream != H0->stream) return fail(SG_EINVAL, "sg_run_group: handle %d is bound to another stream", k);
        for (uint8_t v : H->started)
            if (!v) return fail(SG_ESTATE, "sg_run_group: a replica of handle %d has no start", k);
        for (int32_t j = 0; j < k; ++j)
            if (hs[j] == H) return fail(SG_EINVAL, "sg_run_group: handle %d given twice", k);
    }
    hipStream_t st = H0->stream;
    // start energies left out by sg_init_spins: the queue kernel continues from them
    for (int32_t k = 0; k < count; ++k)
        if ((e = ensure_energy(hs[k])) != SG_OK) return e;
    uint8_t* scr = (uint8_t*)dev_scratch;
    // replica states stay in each handle's workspace: a table entry's rep_base
    // is the offset, in RepState units, of its replica 0 from the first
    // handle's state array (all workspaces are 256-byte aligned)
    sg::RepState* rs0 = H0->reps();
    std::vector<sg::InstTab> tab;
    std::vector<int32_t> ctab;
    std::vector<sg::QueueItem> items;
    std::vector<int32_t> nsz;
    tab.reserve((size_t)g.ninst);
    ctab.reserve((size_t)g.nctab);
    items.reserve((size_t)g.nitems);
    for (int32_t k = 0; k < count; ++k) {
        const sg_ctx* H = hs[k];
        for (const HostInst& q : H->insts) {
            sg::InstTab T{};
            T.I = H->view(q);
            T.spins = H->at<int8_t>(q.off_spins);
            T.spin_stride = (int64_t)q.spin_stride;
            const intptr_t d = (intptr_t)((const uint8_t*)(H->reps() + q.rep_base) - (const uint8_t*)rs0);
            T.rep_base = (int64_t)(d / (intptr_t)sizeof(sg::RepState));
            T.C = q.C;
            T.ctab_off = (int32_t)ctab.size();
            T.nbr_words = (int32_t)q.nbr.size();
            T.tri_words = (int32_t)q.ta.size();
            T.eterm = H->at<uint32_t>(q.off_eterm);
            T.n_eh = q.n_eh;
            T.n_ee = q.n_ee;
            T.n_et = q.n_et;
            for (int32_t c = 0; c <= q.C; ++c) ctab.push_back(q.colour_slice[c]);
            const int32_t gi = (int32_t)tab.size();
            tab.push_back(T);
            nsz.push_back(q.n);
            for (int32_t r = 0; r < q.R; ++r) items.push_back(sg::QueueItem{gi, r});
        }
    }
    // largest items first; those above the wavefront size run on whole workgroups
    std::stable_sort(items.begin(), items.end(),
                     [&](const sg::QueueItem& a, const sg::QueueItem& b) { return nsz[a.inst] > nsz[b.inst]; });
    int n_big = 0, nmax_big = 0, nmax_small = 0;
    for (const sg::QueueItem& it : items) {
        const int n = nsz[it.inst];
        if (n > H0->queue_wave_max_n) {
            ++n_big;
            nmax_big = std::max(nmax_big, n);
        } else {
            nmax_small = std::max(nmax_small, n);
        }
    }
    const int wave_lds = (nmax_small + 15) / 16 * 16;
    size_t lds = std::max<size_t>((size_t)nmax_big, (size_t)wave_lds * 16);
    lds = std::max<size_t>((lds + 15) / 16 * 16, 16);
    if (lds > kLdsBudget) return fail(SG_EINVAL, "sg_run_group: an item needs %zu bytes of LDS", lds);
    int grid = H0->queue_grid;
    if (grid <= 0) grid = sg::queue_max_blocks(lds);
    if (grid <= 0) grid = 256;
    grid = std::min<int>(grid, (int)items.size());
    SG_HIP(hipMemcpyAsync(scr + g.off_tab, tab.data(), tab.size() * sizeof(sg::InstTab), hipMemcpyHostToDevice, st),
           "upload group table");
    SG_HIP(hipMemcpyAsync(scr + g.off_ctab, ctab.data(), ctab.size() * 4, hipMemcpyHostToDevice, st),
           "upload group colour table");
    SG_HIP(hipMemcpyAsync(scr + g.off_items, items.data(), items.size() * sizeof(sg::QueueItem),
                          hipMemcpyHostToDevice, st),
           "upload group items");
    SG_HIP(sg::launch_fill_u32(scr + g.off_cnt, 16, 0u, st), "fill kernel");
    SG_HIP(sg::launch_fill_u32(scr + g.off_stats, sizeof(sg::CallStats) / 4, 0u, st), "fill kernel");
    SG_HIP(hipEventRecord(H0->evh0, st), "event record");
    if (p->max_sweeps > 0)
        SG_HIP(sg::launch_queue(reinterpret_cast<sg::InstTab*>(scr + g.off_tab),
                                reinterpret_cast<int32_t*>(scr + g.off_ctab),
                                reinterpret_cast<sg::QueueItem*>(scr + g.off_items), n_big, (int)items.size(),
                                reinterpret_cast<uint32_t*>(scr + g.off_cnt), wave_lds, lds, grid, rs0,
                                reinterpret_cast<sg::CallStats*>(scr + g.off_stats), p->max_sweeps, p->seed, p->rule,
                                p->until_converged, st),
               "queue kernel");
    SG_HIP(hipEventRecord(H0->evh1, st), "event record");
    sg::CallStats cs{};
    SG_HIP(hipMemcpyAsync(&cs, scr + g.off_stats, sizeof cs, hipMemcpyDeviceToHost, st), "stats copy");
    std::vector<std::vector<sg::RepState>> reps;
    if (unconverged) {
        reps.resize((size_t)count);
        for (int32_t k = 0; k < count; ++k) {
            reps[(size_t)k].resize((size_t)hs[k]->total_reps);
            SG_HIP(hipMemcpyAsync(reps[(size_t)k].data(), hs[k]->reps(), reps[(size_t)k].size() * sizeof(sg::RepState),
                                  hipMemcpyDeviceToHost, st),
                   "state copy");
        }
    }
    SG_HIP(hipStreamSynchronize(st), "stream sync");  // the host tables above are released on return
    if (unconverged)
        for (int32_t k = 0; k < count; ++k) {
            int32_t c = 0;
            for (const sg::RepState& r : reps[(size_t)k]) c += r.converged ? 0 : 1;
            unconverged[k] = c;
        }
    float hms = 0.f;
    if (hipEventElapsedTime(&hms, H0->evh0, H0->evh1) != hipSuccess) {
        (void)hipGetLastError();
        hms = 0.f;
    }
    if (stats) {
        stats->attempts = (int64_t)cs.attempts;
        stats->flips = (int64_t)cs.flips;
        stats->sweeps_max = (int64_t)cs.sweeps_max;
        stats->n_unconverged = (int32_t)cs.unconverged;
        stats->schedule_used = SG_SCHED_QUEUE;
        stats->kernel_ms = hms;
    }
    if (p->until_converged && cs.unconverged) {
        fail(SG_ENOTCONV, "%llu replicas did not converge within %d sweeps", (unsigned long long)cs.unconverged,
             p->max_sweeps);
        return SG_ENOTCONV;
    }
    return SG_OK;
}

sg_status sg_philox_word0(const void* dev_ctr, void* dev_out, int64_t count, uint64_t seed, void* hip_stream)
{
    if (count < 0) return fail(SG_EINVAL, "count must be >= 0");
    if (count > 0 && (!dev_ctr || !dev_out)) return fail(SG_EINVAL, "null device pointer");
    if (((uintptr_t)dev_ctr & 3) || ((uintptr_t)dev_out & 3)) return fail(SG_EINVAL, "pointers must be 4-byte aligned");
    hipStream_t st = (hipStream_t)hip_stream;
    SG_HIP(sg::launch_philox_word0((const uint32_t*)dev_ctr, (uint32_t*)dev_out, count, seed, st), "philox kernel");
    SG_HIP(hipStreamSynchronize(st), "stream sync");
    return SG_OK;
}

sg_status sg_free(sg_handle H)
{
    if (!H) return SG_OK;
    if (H->ev0) (void)hipEventDestroy(H->ev0);
    if (H->ev1) (void)hipEventDestroy(H->ev1);
    if (H->evh0) (void)hipEventDestroy(H->evh0);
    if (H->evh1) (void)hipEventDestroy(H->evh1);
    if (H->cap_stream) (void)hipStreamDestroy(H->cap_stream);
    if (H->pin) (void)hipHostFree(H->pin);
    delete H;
    return SG_OK;
}

}  // extern "C"
