/*
 * sg.h -- C-ABI of the MI355X (gfx950) spin-glass local-search library.
 *
 * The library minimises the hyper-Ising energy of García & Markov
 * ("High-performance Energy Minimization in Spin-glasses with Applications
 * to Adiabatic Quantum Computing"), Sec. II eq. (1) extended by Sec. VI
 * eq. (5) to couplings over three spins:
 *
 *   E(s) = - sum_{edges (i,j)} J_ij s_i s_j - sum_i h_i s_i
 *          - sum_{triples (i,j,k)} K_ijk s_i s_j s_k ,     s_i in {-1,+1}
 *
 * with every undirected edge and every triple counted once, by single-spin
 * moves (Sec. IV): the move of spin i changes the energy by
 * dE_i = 2 s_i f_i, f_i = h_i + sum_j J_ij s_j + sum_(j,k) K_ijk s_j s_k
 * (its gain, in the paper's words, is -dE_i).  Moves are applied in
 * colour-ordered parallel sweeps: the spins are split into colour classes of
 * a proper colouring of the primal graph (edges plus the three pairs of each
 * triple), colours are visited in ascending order and all spins of one
 * colour are decided and flipped at once.  Because no energy term holds two
 * spins of one colour, this equals visiting the spins of the colour one at a
 * time, so every result is that of a sequential descent.  Random starts are
 * uniform (Sec. IV); a run stops when a sweep flips nothing (the stopping
 * rule of Sec. IV, Fig. 3) or after a fixed number of sweeps; independent
 * restarts keep the best (Sec. IV, Sec. V).
 *
 * Randomness: Philox4x32-10 (Salmon et al., SC'11), key = seed (low word,
 * high word), counter = (external spin index, sweep index or 0xFFFFFFFF for
 * the start, instance_id, restart); bit 0 of output word 0 is used.  The
 * sweep index is the replica's absolute sweep count, so splitting a run over
 * several sg_run_sweeps calls gives the same result as one call.
 *
 * All arithmetic is integer: couplings, fields and hyper-couplings are
 * int32 at this boundary, energies and counters int64; every result is
 * exact and reproducible bit for bit.
 *
 * Memory: the library allocates no device memory.  The caller provides one
 * device buffer of sg_workspace_bytes() bytes (for example a torch uint8
 * tensor) and a HIP stream; every kernel runs on that stream.  Host arrays
 * passed in are copied; host output buffers are written before return.
 * A handle is not thread-safe.  All functions return an sg_status; on error
 * sg_last_error() holds a message (thread-local).
 */
#ifndef SG_H
#define SG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sg_status;
enum {
    SG_OK = 0,
    SG_ENOTCONV = 1,   /* warning: until_converged and some replica hit the sweep cap */
    SG_EINVAL = -1,    /* invalid argument or instance (message says which) */
    SG_ERANGE = -2,    /* a value or size outside what the kernels represent */
    SG_ENOMEM = -3,    /* workspace smaller than sg_workspace_bytes(), or host allocation failed */
    SG_EDEVICE = -4,   /* a HIP call failed (message holds the HIP error string) */
    SG_ESTATE = -5     /* call out of order (run or read before bind / init) */
};

/* Acceptance rule of a move with energy change dE. */
enum {
    SG_RULE_GREEDY = 0,      /* flip iff dE < 0 */
    SG_RULE_GREEDY_TIE = 1,  /* also flip when dE == 0 and the sweep's RNG bit is 1 */
    /* The paper's pass-based local search with hill-climbing (Sec. IV,
     * Fig. 3) instead of the colour sweep: a "sweep" is one pass.  From the
     * replica's state SP*, n times the unlocked spin of largest gain -dE
     * (lowest spin index among equal gains) is moved, even at negative gain,
     * and locked; the state of strictly lowest energy seen in the pass becomes
     * SP*.  until_converged: stop after the first pass that leaves the energy
     * unchanged (it counts).  flips counts the moves kept (the best prefix of
     * each pass); attempts = passes x n.  Deterministic (no RNG).  Instances
     * of more than 4096 spins need the knob fm_slots (set before sg_bind:
     * that many replicas run at once, each with ~9 bytes of device scratch per
     * spin in the workspace) and at most 2^24 - 1 spins (else SG_EINVAL);
     * both forms; runs under SG_SCHED_AUTO or SG_SCHED_FM only. */
    SG_RULE_FM = 2
};

/* Execution schedules.  Every schedule computes the same result bit for bit;
 * they differ only in how the sweeps are mapped onto the GPU. */
enum {
    SG_SCHED_AUTO = -1,        /* pick per instance from the tuned table */
    SG_SCHED_PHASE = 0,        /* one kernel launch per colour phase per instance */
    SG_SCHED_GRAPH = 1,        /* SG_SCHED_PHASE captured in HIP graphs of several sweeps */
                               /* 2 is reserved */
    SG_SCHED_LATTICE = 3,      /* lattice instances: LDS-resident tiles, halo exchange */
    SG_SCHED_BLOCK = 4,        /* one workgroup per instance, structure and replicas in LDS */
    SG_SCHED_QUEUE = 5,        /* persistent batched: work queue of uneven instances */
    SG_SCHED_FM = 6,           /* SG_RULE_FM: one wavefront per replica */
    SG_SCHED_FIELDS = 7,       /* SG_SCHED_PHASE over local fields kept in the workspace and
                                  updated by the flips (knob "fields" = 1 before sg_bind) */
    SG_SCHED_DENSE = 8         /* handles from sg_load_dense: one lane per replica */
};

typedef struct sg_ctx* sg_handle;

/* One instance.  Arrays are host memory owned by the caller and copied by
 * sg_load_instance.
 *   n            number of spins, >= 1
 *   m, ei, ej, J undirected couplings (ei[k], ej[k], J[k]); ei != ej, no pair
 *                twice (in either orientation), indices in [0, n)
 *   h            n fields, or NULL for all zero
 *   t, tri, K    3-spin hyper-couplings: tri[3k..3k+2] three distinct spins,
 *                no set of three twice, coefficient K[k]
 *   colour       n colours forming a proper colouring of the primal graph,
 *                or NULL: first-fit colouring over increasing spin index
 *                (spin i takes the smallest colour not used by a primal
 *                neighbour j < i)
 *   dims         lattice hint: {Lx, Ly, Lz} of a periodic hypercubic lattice
 *                with row-major site index (x slowest) and the +axis bond of
 *                every site, or {Lx, Ly, 0} in 2-D; all zero = general
 *                graph.  When given, the edge list must be exactly that
 *                lattice (checked) and SG_SCHED_LATTICE becomes available.
 *   instance_id  RNG key word of the instance; keep it stable across
 *                batching and serving to reproduce results
 *   restarts     independent replicas of this instance, >= 1
 * Values: any int32 coupling, field and hyper-coupling.  SG_ERANGE only when
 * a spin's |h_i| + sum_j |J_ij| + sum |K| exceeds 2^31 - 1 (its local field
 * would not fit int32), when sum|J| + sum|h| + sum|K| exceeds 2^63 - 1 (an
 * energy would not fit int64), or when n exceeds 2^30.  How the library
 * stores an instance (packed 8-bit coefficients and 24-bit indices, or a wide
 * form for larger values, sizes and restart counts) is invisible here: every
 * call accepts both and gives the same results; under GREEDY and
 * GREEDY_TIE the wide form runs on SG_SCHED_PHASE and SG_SCHED_GRAPH
 * (SG_SCHED_AUTO picks them), and SG_RULE_FM runs it one wavefront per
 * replica. */
typedef struct {
    int32_t n;
    int64_t m;
    const int32_t* ei;
    const int32_t* ej;
    const int32_t* J;
    const int32_t* h;
    int64_t t;
    const int32_t* tri;
    const int32_t* K;
    const int32_t* colour;
    int32_t dims[3];
    uint32_t instance_id;
    int32_t restarts;
} sg_instance_desc;

/* Parameters of one sg_run_sweeps call.
 *   seed             Philox key
 *   rule             SG_RULE_*
 *   max_sweeps       sweeps this call may perform per replica (>= 0)
 *   until_converged  1: a replica stops after its first sweep with no flip
 *                    (that sweep counts) and stays frozen until it is
 *                    restarted; 0: exactly max_sweeps sweeps per replica
 *   schedule         SG_SCHED_*; a schedule the instance cannot use gives
 *                    SG_EINVAL */
typedef struct {
    uint64_t seed;
    int32_t rule;
    int32_t max_sweeps;
    int32_t until_converged;
    int32_t schedule;
} sg_run_params;

/* Totals of one sg_run_sweeps call over all replicas of the handle.
 *   attempts       sum over replicas of (sweeps performed) x n
 *   flips          moves applied
 *   sweeps_max     most sweeps performed by one replica
 *   n_unconverged  replicas not converged at return (until_converged only)
 *   kernel_ms      device time of the call's sweep kernels (HIP events) */
typedef struct {
    int64_t attempts;
    int64_t flips;
    int64_t sweeps_max;
    int32_t n_unconverged;
    int32_t schedule_used;
    double kernel_ms;
} sg_run_stats;

/* Per-instance facts after loading. */
typedef struct {
    int32_t n;
    int32_t colours;       /* number of colour classes */
    int64_t m;
    int64_t t;
    int32_t restarts;
    int32_t lattice;       /* 1 if the lattice schedule can run this instance */
    int64_t replica_base;  /* index of replica 0 of this instance in handle order */
} sg_instance_info;

/* Validate and pack `count` instances into one handle (a batch when
 * count > 1).  An instance is the spin glass of Sec. II (couplings J_ij on the
 * edges of a graph and fields h_i, energy eq. (1)) with the three-spin
 * couplings of Sec. VI eq. (5); the problem solved is Sec. II's ground-state
 * search (find spins that minimise E).  Host-only: needs no GPU.  Errors:
 * SG_EINVAL (message names the instance and the problem), SG_ERANGE,
 * SG_ENOMEM. */
sg_status sg_load_instance(const sg_instance_desc* descs, int32_t count, sg_handle* out);

/* Dense hyper-Ising instance (Sec. VI eq. (5)): couplings over any set of
 * spins, such as the factoring hypergraphs of Sec. VI eqs. (6)-(8), whose
 * terms reach four spins and whose coefficients exceed the int8 / int32
 * ranges of sg_instance_desc.  Host arrays, copied by sg_load_dense.
 *   n            1..64 spins
 *   nterms       number of terms (>= 0)
 *   mask         member set of every term: bit i = spin i; non-empty, only
 *                bits below n, no set twice
 *   coef         coefficient of every term:
 *                E(s) = -sum_t coef[t] prod_{i in mask[t]} s_i
 *                (a one-spin term is a field)
 *   instance_id, restarts  as in sg_instance_desc
 * Limit: sum_t |coef[t]| < 2^62 (SG_ERANGE beyond), so energies and gains
 * are exact int64.  The colour sweep orders spins by the first-fit colouring
 * of the graph joining any two spins that share a term. */
typedef struct {
    int32_t n;
    int64_t nterms;
    const uint64_t* mask;
    const int64_t* coef;
    uint32_t instance_id;
    int32_t restarts;
} sg_dense_desc;

/* Validate and pack `count` dense instances into one handle.  The handle
 * takes every other call of this interface: sg_init_spins (same start rule),
 * sg_set_spins, sg_run_sweeps (SG_RULE_GREEDY, SG_RULE_GREEDY_TIE or
 * SG_RULE_FM under SG_SCHED_AUTO or SG_SCHED_DENSE; the same stopping rule
 * and counters), sg_energy, sg_replica_counters, sg_spins_out(_batch),
 * sg_best.  Host-only.  Errors: SG_EINVAL (message names the instance and
 * the problem), SG_ERANGE, SG_ENOMEM. */
sg_status sg_load_dense(const sg_dense_desc* descs, int32_t count, sg_handle* out);

/* Exact ground state by branch-and-bound (Sec. III) on the host CPU: no GPU
 * and no handle.  Spins are assigned in breadth-first order of the primal
 * graph; a partial assignment is pruned when its lower bound (eq. (2) plus
 * 2|c| for every fully assigned term that is unsatisfied, eqs. (3)-(4)) reaches
 * the best energy held, or when a spin whose neighbourhood is fully assigned
 * could be flipped to lower the energy (Lemma 2 with one-spin changes) or to
 * keep it while holding the value tried second.
 *   d           one instance (dims, colour and restarts are ignored)
 *   seed_spins  n spins +-1 (external order) whose energy seeds the bound and
 *               whose values are tried first, e.g. the best restart of
 *               sg_run_sweeps; or NULL
 *   spins_out   n spins: a ground state (the seed when nothing is lower)
 *   E_out       its energy
 *   nodes_out   assignments made by the search (may be NULL)
 *   max_nodes   budget (0 = none); when reached the call returns SG_ENOTCONV
 *               with the best state found so far, not proven optimal
 * The search takes exponential time in the worst case: the paper reports
 * about 100 spins as its practical limit on lattices.  At most 4096 spins. */
sg_status sg_exact_ground_state(const sg_instance_desc* d, const int8_t* seed_spins, int8_t* spins_out,
                                int64_t* E_out, int64_t* nodes_out, int64_t max_nodes);

/* Device bytes the handle needs: packed coupling structure, spins of every
 * replica, per-replica counters and scratch.  Host-only. */
sg_status sg_workspace_bytes(sg_handle h, uint64_t* bytes);

/* Facts about instance `inst` (colour count, replica offset, ...); the
 * colouring actually used is written to colour_out (n entries, external
 * order) when not NULL.  Host-only. */
sg_status sg_instance_info_get(sg_handle h, int32_t inst, sg_instance_info* info,
                               int32_t* colour_out);

/* Bind caller-owned device memory (>= sg_workspace_bytes, 256-byte aligned)
 * and a HIP stream (hipStream_t, NULL = default stream) to the handle, and
 * upload the coupling structure: the instance of Sec. II eq. (1) / Sec. VI
 * eq. (5) and room for the replicas' spin configurations, the state the local
 * search of Sec. IV (Fig. 3) works on; the paper itself defines no memory
 * layout.  The memory must stay allocated while the
 * handle uses it; binding again moves the handle (state is not kept).  The
 * first sg_bind of a handle also allocates 64 KiB of pinned host memory
 * (hipHostMalloc, released by sg_free), through which the later calls read
 * their small results back without a synchronisation per copy.
 * Errors: SG_ENOMEM if too small, SG_EINVAL if misaligned, SG_EDEVICE. */
sg_status sg_bind(sg_handle h, void* dev_ptr, uint64_t bytes, void* hip_stream);

/* Size of the library's static device workspace used by sg_bind_noalloc. */
#define SG_NOALLOC_MAX_BYTES (64ull << 20)

/* sg_bind without caller memory, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  Binds the handle to a workspace of
 * SG_NOALLOC_MAX_BYTES bytes that the library holds in a statically
 * allocated device array (one per GPU, held until the process ends) and to a
 * HIP stream, and uploads the coupling structure, as sg_bind does.  Allocates
 * no device memory (no hipMalloc, no allocating library routine; the
 * handle's HIP timing events are created on its first bind, as by sg_bind)
 * and no pinned host memory: a handle first bound this way reads its results
 * back through pageable copies, one synchronisation each.  Every
 * handle bound this way on one GPU shares that array, which keeps the last
 * user's contents: binding another handle replaces the first one's structure
 * and state (use the first one again only after binding it again), and calls
 * that overlap on one GPU race.  The caller still passes inputs (the loaded
 * handle) and reads outputs into host buffers as with sg_bind.  Errors:
 * SG_ENOMEM when sg_workspace_bytes exceeds SG_NOALLOC_MAX_BYTES, SG_EDEVICE,
 * and those of sg_bind. */
sg_status sg_bind_noalloc(sg_handle h, void* hip_stream);

/* Draw the random start of every replica (Sec. IV: uniform), compute its
 * energy (or leave it to the run that follows, see the "defer_energy" knob
 * of sg_tune), reset sweeps, flips and converged.  Enqueued on the bound
 * stream (returns without waiting for it).  Errors: SG_ESTATE before bind. */
sg_status sg_init_spins(sg_handle h, uint64_t seed);

/* Set replica r of instance inst to host spins s (n int8 values, each +1 or
 * -1, external order) and reset its counters: the starting configuration of
 * the local search (Sec. IV, Fig. 3's input), given instead of drawn; its
 * energy is eq. (1) / eq. (5) of these spins.  Errors: SG_EINVAL for a value
 * other than +-1 or an index out of range; SG_ESTATE before bind. */
sg_status sg_set_spins(sg_handle h, int32_t inst, int32_t r, const int8_t* s);

/* Run colour-ordered sweeps on every replica that is not frozen (enqueued
 * on the bound stream; returns after the stream has finished them): the
 * single-spin moves of Sec. IV with their gains -dE_i (dE_i = 2 s_i f_i), the
 * three-spin terms entering the gains as in Sec. VI, and the stopping rule of
 * Fig. 3 (a pass that brings no improvement ends the search).
 * stats may be NULL.  Returns SG_ENOTCONV when until_converged and a
 * replica hit max_sweeps.  Errors: SG_ESTATE before sg_init_spins or
 * sg_set_spins of every replica, SG_EINVAL for bad parameters or a schedule
 * the handle cannot use, SG_EDEVICE for a HIP failure or a lattice tile
 * kernel whose wait for a neighbour tile timed out (the replica state is then
 * undefined: start again with sg_init_spins). */
sg_status sg_run_sweeps(sg_handle h, const sg_run_params* p, sg_run_stats* stats);

/* Continuous batching: one sg_run_sweeps step over the replicas of `count`
 * handles at once, in a single launch of the persistent queue kernel, so
 * that requests loaded and started at different times share the GPU launch
 * by launch (a serving loop calls it repeatedly with a bounded max_sweeps and
 * lets finished handles leave and new ones join between calls).  Each
 * replica follows exactly the rules of sg_run_sweeps (Sec. IV moves, the
 * stopping rule of Fig. 3, the absolute sweep count in the RNG counter), so
 * its result does not depend on the other handles of the group, on how many
 * calls its sweeps are split over, or on the schedule.
 *   hs, count      distinct bound handles, all bound to the same stream (the
 *                  launch runs on it), every replica started; every instance
 *                  at most 150000 spins in the packed form (sg_query
 *                  "queue_ok" = 1), no dense handles
 *   p              rule SG_RULE_GREEDY or SG_RULE_GREEDY_TIE, schedule
 *                  SG_SCHED_AUTO or SG_SCHED_QUEUE
 *   dev_scratch    caller-owned device memory of at least
 *                  sg_group_scratch_bytes() bytes, 256-byte aligned (the
 *                  group's instance table and work list)
 *   unconverged    host array of `count` entries or NULL: replicas of each
 *                  handle not converged after the call
 *   stats          totals over the group, or NULL
 * Returns after the stream has finished.  SG_ENOTCONV as sg_run_sweeps.
 * Errors: SG_EINVAL (a handle that cannot join, another stream, bad
 * parameters), SG_ESTATE, SG_ENOMEM (scratch too small), SG_EDEVICE. */
sg_status sg_group_scratch_bytes(const sg_handle* hs, int32_t count, uint64_t* bytes);
sg_status sg_run_group(const sg_handle* hs, int32_t count, const sg_run_params* p, void* dev_scratch,
                       uint64_t scratch_bytes, int32_t* unconverged, sg_run_stats* stats);

/* Energies of all replicas in handle order (sum over instances of
 * restarts entries): E(s) of Sec. II eq. (1) with the three-spin terms of
 * Sec. VI eq. (5), every edge and triple once, exact in int64.  recompute = 0: the tracked energy (start energy plus
 * the dE of every applied move); recompute = 1: a fresh evaluation of the
 * energy from the current spins. */
sg_status sg_energy(sg_handle h, int64_t* E, int32_t recompute);

/* Per-replica counters in handle order (any pointer may be NULL): sweeps
 * performed since the last start, moves applied, converged flag. */
sg_status sg_replica_counters(sg_handle h, int64_t* sweeps, int64_t* flips, int8_t* converged);

/* Spins of replica r of instance inst, n int8 values in external order: the
 * configuration the search reached (Fig. 3's output, Sec. II's solution of
 * the ground-state problem when it is a ground state). */
sg_status sg_spins_out(sg_handle h, int32_t inst, int32_t r, int8_t* s);

/* Spins of restarts r0 .. r0+count-1 of instance inst: count x n int8 values,
 * restart-major, each in external order.  Errors: SG_EINVAL for a range
 * outside [0, restarts). */
sg_status sg_spins_out_batch(sg_handle h, int32_t inst, int32_t r0, int32_t count, int8_t* s);

/* Multi-start result per instance (Sec. IV: keep the best start): lowest
 * tracked energy over its restarts, lowest restart index on ties.  E_best and
 * r_best have one entry per instance; either may be NULL. */
sg_status sg_best(sg_handle h, int64_t* E_best, int32_t* r_best);

/* A whole multi-start search in one call (Sec. IV: random starts, the local
 * search, keep the best): sg_init_spins(h, p->seed), then sg_run_sweeps(h, p,
 * stats), then sg_best(h, E_best, r_best), with the same results, replica
 * states and statuses as those three calls.  When every instance is a
 * lattice that one workgroup holds (at most lattice_wg_max_n spins, lattice
 * hint given) and the run would take SG_SCHED_LATTICE, the start, the sweeps
 * and the replica energies run as one kernel launch per instance and the call
 * synchronises once; otherwise it makes the three calls.  Errors: those of
 * the three calls (SG_ENOTCONV after every output is written). */
sg_status sg_solve(sg_handle h, const sg_run_params* p, sg_run_stats* stats, int64_t* E_best, int32_t* r_best);

/* Tuning knobs of the schedules; results never depend on them.
 *   "lattice_k"          colour phases between halo exchanges of the lattice
 *                        tile schedule (1..16, default 4)
 *   "lattice_max_tiles"  cap on tiles per replica (0 = as many as fit)
 *   "lattice_wg_max_n"   largest lattice run with one workgroup per replica
 *   "block_rg"           restarts per workgroup of the block schedule
 *                        (64, 128, 256; 0 = 64, the fastest measured)
 *   "block_groups"       restarts per workgroup of the block schedule in
 *                        units of block_rg: its slots take the next restart
 *                        as replicas stop (0 = up to 4, fewer when the
 *                        workgroups would not fill the GPU; at most 64)
 *   "block_bits"         1: GREEDY on the block schedule uses the bit-sliced
 *                        kernel (32 restarts per word) for instances of at
 *                        most 2048 spins whose coefficients are at most 15
 *                        in magnitude and sum to at most 255 per spin; 0:
 *                        always the byte kernel (default 1)
 *   "bits_groups"        most groups of 32 restarts per bit-sliced workgroup
 *                        (2, 4, 8, 16; default 8)
 *   "defer_energy"       1: sg_init_spins leaves out the start energy of
 *                        instances that SG_SCHED_AUTO would run on a kernel
 *                        that computes the energies of the final spins
 *                        itself: the bit-sliced block kernel, the bit-plane
 *                        lattice tile kernel, or the queue kernel (from the
 *                        last sweep of a converged replica).  When a run
 *                        leaves some replica without (a sweep cap, another
 *                        kernel), the energies are computed after it.  Any other reader
 *                        (sg_energy, sg_best, another rule or schedule, a
 *                        run without until_converged) first computes them.
 *                        0: always at the start (default 1; results are the
 *                        same)
 *   "fm_waves"           most wavefronts per SG_RULE_FM workgroup (0 = 16);
 *                        among the sizes that fit LDS the one with the most
 *                        wavefronts resident per compute unit is used
 *   "fm_key32"           1: SG_RULE_FM picks moves on 32-bit keys when every
 *                        gain is below 2^19 in magnitude; 0: 64-bit keys
 *                        (default 1)
 *   "fm_slots"           replicas of instances beyond 4096 spins that
 *                        SG_RULE_FM runs at once (0 = none: such instances
 *                        are rejected); sizes the workspace (before sg_bind)
 *                        with ~9 bytes per spin of the largest such instance
 *                        per slot, plus each such instance's term rows in
 *                        external order; more slots hide more memory latency
 *   "fm_lanes"           1: SG_RULE_FM runs one replica per lane for every
 *                        instance of at most 1024 spins whose per-spin sum
 *                        |h|+sum|J|+sum|K| is at most 127 (the others one
 *                        replica per wavefront); 0: one replica per wavefront
 *                        throughout (default 1; results are the same).  The
 *                        per-spin term lists of those instances are part of
 *                        the workspace (about 4 words per spin and 1 per
 *                        coupling incidence); 0 set before sg_bind leaves
 *                        them out, and 1 after such a bind is SG_EINVAL
 *   "fm_lane_restarts"   restarts handed to one wavefront of the lane kernel,
 *                        which refills its lanes from them as replicas finish
 *                        (0 = the largest multiple of 64 that still gives
 *                        every resident wavefront one; else a multiple of 64)
 *   "block_min_restarts" SG_SCHED_AUTO uses the block schedule for instances
 *                        with at least this many restarts (default 32)
 *   "queue_wave_max_n"   queue items with at most this many spins run one per
 *                        wavefront, larger ones on a whole workgroup (512)
 *   "queue_grid"         workgroups of the persistent queue launch (0 = all
 *                        that fit co-resident)
 *   "queue_min_items"    SG_SCHED_AUTO uses the queue schedule when the
 *                        handle has at least this many queue items (32)
 *   "graph_sweeps"       sweeps per captured HIP graph of SG_SCHED_GRAPH
 *                        (1..1024, default 32)
 *   "auto_graph"         1: SG_SCHED_AUTO records the per-phase launches of the
 *                        instances it would run on SG_SCHED_PHASE in HIP graphs
 *                        (SG_SCHED_GRAPH); 0: plain launches (default 0; the
 *                        autotuner of the Python package sets it where
 *                        graphs measure faster)
 *   "lattice_msc"        1: tile lattices whose bonds are all +-1 and whose
 *                        fields satisfy |h| <= 2 with the bit-plane kernel
 *                        (32 sites of a colour per lane word); 0: byte kernel
 *   "msc_k"              halo width of the bit-plane kernel (0 = chosen by
 *                        its cost model, else 1..62)
 *   "lattice_conv_chunk" most sweeps of one bit-plane launch under
 *                        until_converged (1..16384, default 16384); a call
 *                        that needs more runs several launches
 *   "fields"             1: the workspace also holds each replica's local
 *                        fields (4 bytes per spin per replica) and
 *                        SG_SCHED_FIELDS becomes available (SG_SCHED_AUTO
 *                        then uses it where it would use SG_SCHED_PHASE);
 *                        changes sg_workspace_bytes, so it must be set
 *                        before sg_bind (SG_EINVAL after)
 * Unknown key or value out of range: SG_EINVAL. */
sg_status sg_tune(sg_handle h, const char* key, int64_t value);

/* Read a knob, or one of "last_tiles" (Px*10^6 + Py*10^3 + Pz of the last
 * lattice tile launch), "last_tile_k", "last_msc" (1 when that launch used
 * the bit-plane kernel), "last_model_phase_ns" / "last_model_exchange_ns" /
 * "last_model_phases" / "last_model_exchanges" (the bit-plane tiling's
 * latency model for that launch: mean cost of one colour phase and of one
 * halo exchange, and how many of each the launch holds), "last_bits" (1 when the last block-schedule call
 * used the bit-sliced kernel), "last_key32" (1 when the last SG_RULE_FM call
 * picked moves on 32-bit keys), "last_fm_waves" (its wavefronts per
 * workgroup, 0 when every replica ran one per lane), "last_fm_lanes" (its
 * replicas run one per lane), "last_fm_lane_nr" (its restarts per lane-kernel
 * wavefront), "last_fm_big" (its replicas on the kernel for instances beyond
 * 4096 spins), "energy_pending" (1 while start energies
 * left out by sg_init_spins are not yet computed), "last_queue_grid",
 * "total_replicas", "queue_ok" (1 when every instance can join sg_run_group),
 * "wide_instances" (instances stored in the wide form: a
 * coefficient beyond int8, a spin with |h|+sum|J|+sum|K| >= 2^23 or more than
 * 255 triples, n >= 2^24 or more than 65535 restarts; they run on
 * SG_SCHED_PHASE or SG_SCHED_GRAPH),
 * "instances", "hot_ns" / "hot_launches" (device time, from HIP events on the
 * bound stream, of the last sg_run_sweeps call's sweep kernel launches: the
 * single launch of the lattice, block or queue schedule, or the span of the
 * per-phase launches, and how many launches that span holds). */
sg_status sg_query(sg_handle h, const char* key, int64_t* value);

/* The device generator behind every random start and tie decision, exposed
 * so that it can be checked against published values: word 0 of
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11; ten rounds, key = seed:
 * low word, high word) for `count` counters.
 *   dev_ctr     device memory, 4 x count uint32: counter words 0..3 of each
 *   dev_out     device memory, count uint32 (written)
 *   hip_stream  hipStream_t the kernel runs on (NULL = default stream); the
 *               call returns after the stream has finished it
 * Both buffers are caller-owned and 4-byte aligned.  Errors: SG_EINVAL (bad
 * count, null or misaligned pointer), SG_EDEVICE. */
sg_status sg_philox_word0(const void* dev_ctr, void* dev_out, int64_t count, uint64_t seed, void* hip_stream);

/* Release the handle (not the caller's device memory).  NULL is allowed. */
sg_status sg_free(sg_handle h);

/* Message of the last error on this thread ("" if none). */
const char* sg_last_error(void);

/* Library version string. */
const char* sg_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SG_H */
