// sg_launch.h -- launchers of the library's HIP kernels (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sg_layout.h"

namespace sg {

hipError_t launch_fill_u32(void* p, uint64_t count, uint32_t v, hipStream_t st);
// Energy of every replica of one instance into rs[r].E (out == NULL) or out[r].
hipError_t launch_energy(const InstDev& I, const int8_t* spins, int64_t stride, int R, int64_t* slots,
                         int nslots, RepState* rs, int64_t* out, hipStream_t st);
// out[r] (or rs[r].E when out is null) = sum of slots[r * nslots ...], r < R.
hipError_t launch_reduce_energy(const int64_t* slots, int nslots, int R, RepState* rs, int64_t* out, hipStream_t st);
hipError_t launch_begin(RepState* rs, int R, int64_t* acc, int64_t nacc, hipStream_t st);
// t_rel is relative to *t_base when t_base is not null (graph replays);
// with fields not null the phase reads and maintains the replicas' local
// fields (fstride ints between replicas) instead of summing the couplings.
hipError_t launch_phase(const InstDev& I, int8_t* spins, int64_t stride, RepState* rs, int R, int64_t* acc,
                        int nslots, int slice0, int nslice_c, int t_rel, uint64_t seed, int rule,
                        int until_conv, hipStream_t st, const int32_t* t_base = nullptr, int32_t* fields = nullptr,
                        int64_t fstride = 0);
hipError_t launch_fields(const InstDev& I, const int8_t* spins, int64_t stride, int R, int32_t* fields, int64_t fstride,
                         hipStream_t st);
hipError_t launch_bump(int32_t* t_base, int d, hipStream_t st);
// Fold a call's per-slot accumulators into the replicas (absolute: the slots
// hold shares of the final energy instead of energy changes).
hipError_t launch_end(RepState* rs, int R, const int64_t* acc, int nslots, int T, int until_conv, int64_t n,
                      CallStats* cs, hipStream_t st, bool absolute = false);
hipError_t launch_any_active(const RepState* rs, int R, int T, uint32_t* flag, hipStream_t st);
// Word 0 of Philox4x32-10 of count counters (4 uint32 each) under key seed.
hipError_t launch_philox_word0(const uint32_t* ctr, uint32_t* out, int64_t count, uint64_t seed, hipStream_t st);
hipError_t launch_best(const RepState* rs, const int64_t* rep_base, const int32_t* restarts, int ninst,
                       int64_t* Eb, int32_t* rb, hipStream_t st);

// wide-form instances (sg_wide.hip): one colour phase, and the energy of
// every replica (into rs[r].E, or out[r] when out is not null)
hipError_t launch_wide_phase(const WideDev& I, int8_t* spins, int64_t stride, RepState* rs, int R, int64_t* acc,
                             int nslots, int slice0, int nslice_c, int t_rel, uint64_t seed, int rule, int until_conv,
                             hipStream_t st, const int32_t* t_base = nullptr);
hipError_t launch_wide_energy(const WideDev& I, const int8_t* spins, int64_t stride, int R, int64_t* slots,
                              int nslots, RepState* rs, int64_t* out, hipStream_t st);

// lattice schedules (sg_lattice.hip)
size_t lattice_tiles_lds(const TileGeom& tg, const int L[3], int D);
int lattice_tiles_ns(const TileGeom& tg, const int L[3], int D);  // 0 if the box is too large
int lattice_tiles_max_blocks(const TileGeom& tg, const int L[3], int D);
hipError_t launch_lattice_tiles(const LatticeDev& Lt, const TileGeom& tg, int8_t* canon, int64_t stride,
                                uint64_t* G0, uint64_t* G1, uint32_t* err, RepState* rs, int R,
                                int64_t* acc, int nslots, int T, uint64_t seed, int rule, hipStream_t st);
// exchange words of one copy for a tiling (per replica)
int64_t lattice_tiles_words(const TileGeom& tg, const int L[3]);
// Multi-spin coded tile kernel (lattices with +-1 couplings and |h| <= 2).
size_t lattice_msc_lds(const TileGeom& tg, const int L[3], int D);
bool lattice_msc_geometry_ok(const TileGeom& tg, const int L[3], int D);
int lattice_msc_max_blocks(const TileGeom& tg, const int L[3], int D);
// With scnt (per-sweep tile counters, R x T words, zero on entry) the launch
// runs GREEDY under the stopping rule and a settle kernel then sets each
// replica's lastflip to done + its first sweep without a flip (or done + T).
hipError_t launch_lattice_msc(const LatticeDev& Lt, const TileGeom& tg, int8_t* canon, int64_t stride, uint64_t* G0,
                              uint64_t* G1, uint32_t* err, RepState* rs, int R, int64_t* acc,
                              int nslots, int T, uint64_t seed, int rule, hipStream_t st, uint64_t* scnt = nullptr,
                              int done = 0);
// The paper's pass-based search, one wavefront per replica item.
size_t fm_lds_bytes(int nmax, int waves);
// Workgroups of `waves` wavefronts of the pass kernel with this much LDS
// that fit one compute unit at once.
int fm_max_blocks_per_cu(int waves, size_t lds, bool tri, bool key32);
// stage_cap: LDS bytes after the wavefronts' slices in which a block stages
// its instance's structure when all its items share one instance.
hipError_t launch_fm(const InstTab* tab, const int32_t* ctab, const QueueItem* items, int nitems, int nmax, int waves,
                     int stage_cap, bool tri, bool key32, RepState* rs, CallStats* cs, uint32_t* err, int max_passes,
                     int until_conv, hipStream_t st);
// The pass-based search on instances of more than 4096 spins (packed form,
// term rows FmbRows per instance): one wavefront per slot takes the items
// (replicas) from *counter, zero at launch; per slot slot_spins half-gains,
// move entries and spin bytes and slot_leaves leaf keys; top_cap >= the
// largest instance's ceil(ceil(n / 64) / 64).
hipError_t launch_fm_big(const InstTab* tab, const FmbRows* rows, const QueueItem* items, int nitems,
                         uint32_t* counter, int32_t* half, int32_t* moves, uint64_t* leaf, int8_t* spins,
                         int64_t slot_spins, int64_t slot_leaves, int slots, int top_cap, RepState* rs, CallStats* cs,
                         uint32_t* err, int max_passes, int until_conv, hipStream_t st);
// The pass-based search on one instance in the wide form (at most 4096
// spins), one wavefront per replica of [0, R); rs and spins are the
// instance's own.
hipError_t launch_fm_wide(const WideDev& I, int8_t* spins, int64_t stride, RepState* rs, int R, CallStats* cs,
                          uint32_t* err, int max_passes, int until_conv, hipStream_t st);
// The pass-based search with one replica per lane (instances of at most 1024
// spins whose per-spin sum of |coefficients| is at most 127, with the
// per-spin term rows InstTab::fml): workgroup k runs restarts [r0, r0 + nr)
// of item k's instance on its wavefronts, handing them out through the
// item's pad word, which must be zero at launch, on W wavefronts per
// workgroup.  fml_waves_per_block: the wavefronts of one workgroup for
// instances of up to nmax spins, want (0: one) bounded by four and the LDS
// (0: too large); fml_resident_blocks: such workgroups resident on the device.
// Every instance of one launch has rows of the widths dc (4, 6, 8 or 16
// coupling words) and tt (0, 2, 4 or 6 hyper-couplings) (InstTab::fml_dc,
// fml_tt).
int fml_waves_per_block(int nmax, int want);
int fml_resident_blocks(int nmax, int W, int dc, int tt);
hipError_t launch_fm_lanes(const InstTab* tab, BlockItem* items, int nitems, int nmax, int W, int dc, int tt,
                           RepState* rs, CallStats* cs, uint32_t* err, int max_passes, int until_conv, hipStream_t st);
// Dense hyper-Ising instances: one lane per replica; items are (instance,
// first restart, count <= 64).  rule 0/1: colour sweeps; 2: pass-based search.
hipError_t launch_dense_init(const DenseTab* tabs, const BlockItem* items, int nitems, RepState* rs, uint64_t seed,
                             hipStream_t st);
hipError_t launch_dense_energy(const DenseTab* tabs, const BlockItem* items, int nitems, int64_t* out, hipStream_t st);
hipError_t launch_dense_run(const DenseTab* tabs, const BlockItem* items, int nitems, int nmax, RepState* rs,
                            CallStats* cs, int rule, int max_sweeps, int until_conv, uint64_t seed, hipStream_t st);
// One workgroup per replica of a small lattice.  With a WgSolve the launch is
// a whole solve: it draws each replica's start (seed also keys the start),
// runs the sweeps from sweep 0, and leaves the replica state (exact final
// energy, counters, converged) and the call totals in stats as a start, a run
// and its end kernel would (acc is then unused).  The workgroup that finishes
// last (stats->done reaching done_end, counted over the launches of one
// solve) writes the instance's best restart to best_E / best_r and, when
// stats_out is given, a copy of the call totals there.
struct WgSolve {
    CallStats* stats;
    int64_t* best_E;
    int32_t* best_r;
    CallStats* stats_out;
    unsigned long long done_end;
};
hipError_t launch_lattice_wg(const LatticeDev& Lt, int8_t* canon, int64_t stride, RepState* rs, int R, int64_t* acc,
                             int nslots, int T, uint64_t seed, int rule, int until_conv, hipStream_t st,
                             const WgSolve* solve = nullptr);

// batched schedules (sg_batch.hip)
size_t block_lds_bytes(int n, int nbr_words, int tri_words, int nslices, int C, int RG);
hipError_t launch_block(const InstTab* tab, const int32_t* ctab, const BlockItem* items, int n_items, size_t lds,
                        RepState* rs, CallStats* cs, int RG, int T, uint64_t seed, int rule, int until_conv,
                        hipStream_t st);
// The block schedule under GREEDY with 32 restarts per LDS word (NG groups of
// 32 per workgroup); a finished group computes its restarts' energies.
size_t block_bits_lds_bytes(int n, int nbr_words, int tri_words, int nslices, int C, int NG);
hipError_t launch_block_bits(const InstTab* tab, const int32_t* ctab, const BlockItem* items, int n_items, size_t lds,
                             RepState* rs, CallStats* cs, int NG, int T, int until_conv, hipStream_t st);
int block_bits_max_blocks(size_t lds, int NG);
// Workgroups of the block kernel with this much LDS that fit the GPU at once.
int block_max_blocks(size_t lds);
int queue_max_blocks(size_t lds);
// Start (init) or energy of many replicas of small instances, one lane per
// replica; items (instance, first restart, count <= 64), instances of at most
// 2048 spins.  Without init the energies go to out (or rs when out is null).
// With init, an item whose pad field is nonzero leaves its replicas' E at 0.
hipError_t launch_start_lanes(const InstTab* tab, const BlockItem* items, int nitems, int nmax, bool init,
                              RepState* rs, int64_t* out, uint64_t seed, hipStream_t st);
// Batched start (init: spins drawn by units of 1024 spins, state reset) and
// energy (units of four slices, each summed into part[unit], n_energy
// entries; then the units of each replica segment added into rs[g].E, or
// into out[g] when out is given).
hipError_t launch_start_units(const InstTab* tab, const StartUnit* start_units, int64_t n_start,
                              const StartUnit* energy_units, int64_t n_energy, const EnergySeg* segs, int64_t nsegs,
                              int64_t* part, RepState* rs, int64_t* out, uint64_t seed, bool init, hipStream_t st);
hipError_t launch_queue(const InstTab* tab, const int32_t* ctab, const QueueItem* items, int n_big, int n_items,
                        uint32_t* counters, int wave_lds, size_t lds, int grid, RepState* rs, CallStats* cs, int T,
                        uint64_t seed, int rule, int until_conv, hipStream_t st);

}  // namespace sg
