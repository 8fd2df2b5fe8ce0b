/*
 * emstep.h -- C ABI of the step-based electromagnetic shower transport library
 * for AMD MI355X (gfx950).
 *
 * The library implements the data-parallel hot path described in arXiv
 * 2503.17608 ("Accelerating detector simulations with Celeritas"):
 *
 *   - a step-based transport loop ("Stepping algorithm"): the host runs a
 *     loop of step iterations; each iteration is a sequence of kernels, one
 *     per stepping action, over a fixed array of track slots stored as a
 *     struct of arrays (here with position, direction, energy and key in
 *     one 64-byte record per slot, since every step reads them together);
 *   - secondaries are pushed to a buffer of lightweight track initializers
 *     and vacant slots are filled from it at the start of every iteration;
 *     only the interaction kernels create them (a positron that stops in its
 *     along-step annihilates at rest in the interaction kernels of the same
 *     iteration);
 *   - optional reordering of track slots by next action
 *     ("Reindexing track slots") and optional partitioning of new tracks into
 *     charged / neutral ends of the slot array ("Partitioning track data");
 *   - a cap on field-propagation substeps per iteration after which a track's
 *     step is paused and resumed ("Reducing load imbalance");
 *   - stream-ordered memory operations only ("Asynchronous memory
 *     management");
 *   - on top of the paper's loop: FP32 energies and directions (mixed
 *     precision), continuous batching of events (serving), run-time tuning,
 *     one fused launch for the interaction kernels, and a block-local drain
 *     of the last tracks.
 *
 * The caller's sequence follows the statement of the problem: load geometry,
 * materials and physics tables; push primaries; step until the slots are
 * empty; read back energy deposition.
 *
 * Units: MeV (energies), cm (lengths), g/cm^3 (densities), tesla (field),
 * eV (mean excitation energy only).
 *
 * Conventions for every entry point:
 *   - all functions return ems_status (EMS_OK == 0 on success); no C++
 *     exception crosses this interface; ems_last_error() gives a message for
 *     the calling thread's last failure;
 *   - host pointers are read (or written) before the call returns, and the
 *     caller keeps ownership of them;
 *   - `device_workspace` is device memory owned by the caller (e.g. one torch
 *     uint8 tensor); it must stay allocated until ems_destroy();
 *   - all device work is ordered on the HIP stream given to ems_create();
 *     calls returning results to host memory synchronize that stream.
 */
#ifndef EMSTEP_H
#define EMSTEP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EMS_ABI_VERSION 8u

typedef enum {
    EMS_OK = 0,
    EMS_ERR_INVALID_ARG = -1,  /* bad pointer, size or value */
    EMS_ERR_STATE = -2,        /* call out of order (e.g. push before load) */
    EMS_ERR_CAPACITY = -3,     /* a buffer (initializers, primaries, event rows) is full */
    EMS_ERR_DEVICE = -4,       /* a HIP call failed */
    EMS_ERR_NUMERIC = -5,      /* non-finite value detected */
    EMS_ERR_UNSUPPORTED = -6
} ems_status;

typedef enum { EMS_FP64 = 0, EMS_MIXED = 1 } ems_precision;
/* Track ordering before the along-step and the interaction kernels:
 *   NONE      every kernel runs over all slots and masks by next action;
 *   PARTITION stable counting sort of slot indices by next action (LDS
 *             histogram, scan, stable scatter) at both sort points;
 *   RADIX     the same with the composite key action|particle|material;
 *   QUEUE     PARTITION before the along-step kernels; before the
 *             interaction kernels, the along-step kernels append each
 *             interacting track's slot to its process list (wave-aggregated,
 *             ascending slot order within a wavefront), so no second sort
 *             pass runs. */
/* Paper: "Stepping algorithm" (masking, NONE); "Reindexing track slots" (the others). */
typedef enum { EMS_SORT_NONE = 0, EMS_SORT_PARTITION = 1, EMS_SORT_RADIX = 2, EMS_SORT_QUEUE = 3 } ems_sort_policy;
typedef enum { EMS_GAMMA = 0, EMS_ELECTRON = 1, EMS_POSITRON = 2 } ems_particle;

/* Physics table layout (per material, in this order, 181 nodes each):
 * Compton, photoelectric, pair, Moller, Bhabha, bremsstrahlung macroscopic
 * cross sections [1/cm]; electron range, positron range [cm].  Nodes are at
 * kinetic energies exp(ln(1e-3 MeV) + i ln(10)/20), i = 0..180. */
#define EMS_TABLE_NODES 181
#define EMS_TABLES_PER_MATERIAL 8

typedef struct {
    uint32_t abi_version;      /* must be EMS_ABI_VERSION */
    int32_t precision;         /* ems_precision: FP64, or FP32 energies/directions/tables with FP64 positions */
    uint64_t n_slots;          /* track slots (threads of the state arrays), in [1, 2^30] */
    uint64_t n_initializers;   /* capacity of the secondary initializer buffer */
    uint64_t n_primaries;      /* capacity of the pending-primary buffer */
    uint32_t max_events;       /* tally rows (events resident at once) */
    uint32_t max_slabs;        /* capacity for geometry slabs */
    uint32_t max_materials;    /* capacity for materials */
    int32_t sort_policy;       /* ems_sort_policy, applied before the along-step and interaction kernels
                                  (paper: "Reindexing track slots") */
    int32_t init_partition;    /* 1: new charged tracks fill vacancies from the low end, neutral from the high end
                                  (paper: "Partitioning track data") */
    int32_t max_substeps;      /* field substeps per track per iteration; <= 0 means unlimited
                                  (paper: "Reducing load imbalance") */
    uint64_t seed;             /* Philox key word 0 */
    int32_t block_size;        /* threads per block for the step kernels (multiple of 64, <= 512); 0 = 256 */
    int32_t graph_iterations;  /* iterations captured per HIP graph in ems_run (needs a non-null
                                  stream); 0 = plain launches (paper: "Stepping algorithm", the
                                  launch overhead of the outer loop) */
    int32_t lds_tables;        /* 1: each block of the along-step kernels (which run the pre-step)
                                  and of the drain stages the physics tables in LDS; 0: tables are
                                  read through the caches */
    int32_t streams;           /* 1..4: independent kernels of an iteration (the along-step kernels;
                                  the interaction kernels) run as concurrent branches on up to this
                                  many default-priority streams created by the library (paper:
                                  "Asynchronous memory management", concurrent streams) */
    int32_t msc;               /* 1: charged tracks still in the stack after an along-step are deflected
                                  by multiple scattering: Rayleigh-distributed space angle of Highland
                                  width at the pre-step energy, uniform azimuth (Philox domain 5);
                                  0: no scattering (the physics of the benchmark workloads) */
    int32_t deterministic;     /* 1: secondaries enter the initializer buffer in the order of the
                                  interacting tracks (their positions in the sort permutation, or
                                  their slots when unsorted) instead of the order in which blocks
                                  reach the buffer, so the buffer contents, the slots the fill assigns
                                  and every integer of the state repeat exactly from run to run; the
                                  interaction kernels stage up to 3 records per slot (240 B per slot
                                  more workspace) and two kernels append them after the interactions.
                                  The queue policy (its lists) and the drain (its block-local stacks)
                                  append out of order: they are rejected.  0: block-aggregated appends
                                  (paper: "Stepping algorithm", the deterministic fill of vacancies) */
} ems_options;

typedef struct { double Z, A, density, I_eV; } ems_material;

/* a primary track: `event` is the caller's event id (Philox key word 1) */
typedef struct {
    uint64_t event;
    uint64_t key;              /* track key (Philox counter word 0) */
    int32_t type;              /* ems_particle */
    int32_t slab;              /* slab containing r (on a plane: the slab entered) */
    double T;                  /* kinetic energy [MeV], must be >= the cut */
    double r[3];
    double u[3];               /* unit direction */
} ems_primary;

/* host view of one track slot (debug inject / read) */
typedef struct {
    uint64_t key;
    uint32_t row;              /* tally row of the track's event */
    uint32_t step;             /* completed steps */
    int32_t type;              /* ems_particle, or -1 for a vacant slot */
    int32_t slab;
    double T;
    double nl;                 /* remaining mean free paths, < 0 = to be sampled */
    double r[3];
    double u[3];
} ems_track;

typedef struct {
    double escaped;            /* kinetic energy leaving the stack [MeV] */
    uint64_t n_pair, n_annih, steps;
    uint64_t n_sec[3];         /* secondaries created, by ems_particle */
    uint64_t n_guard;          /* tracks stopped by the step guard */
    uint64_t n_reject_cap;     /* rejection loops that hit their trial cap */
} ems_ledger;

typedef struct {
    uint64_t iterations;       /* step iterations executed so far */
    uint64_t alive;            /* live tracks at the start of the last iteration */
    uint64_t queued;           /* secondary initializers waiting */
    uint64_t pending_primaries;
    uint64_t steps;            /* completed steps of tracks that have finished */
    uint32_t overflow;         /* nonzero: the initializer buffer overflowed (results invalid) */
    uint32_t completed;        /* events completed since creation */
    /* cumulative tracks processed per kernel role: [0] slots handed from a
     * finished track to its secondary, [1] init, [2] pre-steps (run by the
     * along-step kernels), [4] neutral,
     * [5] charged, [6] field along-step (track-iterations), [7..12] Compton,
     * photoelectric, pair, Moller, Bhabha, bremsstrahlung, [13] annihilation
     * at rest, [14] paused field steps, [15] field RK4 evaluations, [16]
     * drain steps */
    uint64_t work[24];
} ems_counters;

typedef struct ems_ctx ems_ctx;

/* Library ABI version (EMS_ABI_VERSION).
 * Paper: no passage (interface versioning). */
uint32_t ems_abi_version(void);

/* Message for the calling thread's most recent failure ("" if none).  The
 * string is owned by the library and valid until the next call.
 * Paper: no passage (error reporting). */
const char* ems_last_error(void);

/* Bytes of device workspace needed for `opt`.  Errors: INVALID_ARG.
 * Paper: "Stepping algorithm" (a fixed array of track slots stored as a struct
 * of arrays, plus the buffer of track initializers); "Asynchronous memory
 * management" (the caller allocates once, stream-ordered). */
ems_status ems_query_workspace(const ems_options* opt, uint64_t* bytes);

/* Create a context on the current HIP device.  `device_workspace` (>= the
 * queried bytes, 256-byte aligned) and `hip_stream` (a hipStream_t, may be
 * NULL for the null stream) are borrowed.  Errors: INVALID_ARG, DEVICE.
 * Paper: "Asynchronous memory management" (all device work ordered on one
 * stream; pinned host buffers for the counters and the staging of primaries). */
ems_status ems_create(const ems_options* opt, void* device_workspace, uint64_t bytes, void* hip_stream,
                      ems_ctx** out);

/* Release the context (not the caller's workspace).
 * Paper: no passage (resource release). */
void ems_destroy(ems_ctx* ctx);

/* Materials (Z, A [g/mol], density, I [eV]); n <= max_materials.
 * Paper: "Stepping algorithm" (the step-limit and interaction actions read
 * per-material data); the physics itself is this library's reading, the paper
 * states none. */
ems_status ems_load_materials(ems_ctx* ctx, const ems_material* m, uint32_t n);

/* Slab stack along z: z_planes[n_slabs + 1] strictly increasing, material
 * index per slab, lateral half width (|x|, |y| <= half_width), uniform field
 * B[3] in tesla.  Outside the stack is a kill region (escape).
 * Paper: "Stepping algorithm" (propagation to boundaries); "Reducing load
 * imbalance" (uniform magnetic field, substepped propagation). */
ems_status ems_load_geometry(ems_ctx* ctx, const double* z_planes, const int32_t* slab_material,
                             uint32_t n_slabs, double half_width, const double B[3]);

/* Build the physics tables on the device from the loaded materials for the
 * production/tracking cut `ecut` [MeV] (the same cut applies to delta rays,
 * bremsstrahlung photons and all tracked particles).  Requires materials.
 * Paper: "Stepping algorithm" (step limit from cross sections and range); the
 * models are this library's reading, the paper states none. */
ems_status ems_build_tables(ems_ctx* ctx, double ecut);

/* Load caller-provided tables instead: `tables` holds
 * [n_materials][EMS_TABLES_PER_MATERIAL][EMS_TABLE_NODES] doubles in the
 * layout described above; copied to the device.
 * Paper: "Stepping algorithm" (as ems_build_tables). */
ems_status ems_load_tables(ems_ctx* ctx, const double* tables, uint32_t n_materials, double ecut);

/* Copy the device tables (FP64) to host `out` (same layout).
 * Paper: no passage (inspection of the loaded tables). */
ems_status ems_read_tables(ems_ctx* ctx, double* out, uint64_t n_doubles);

/* Queue primaries (copied to device).  Each event id is given a tally row on
 * first sight.  Errors: STATE (nothing loaded), INVALID_ARG (bad type, slab,
 * energy below the cut or not finite, direction not unit, position outside
 * the given slab or the lateral walls), CAPACITY (primary buffer or event
 * rows full).  Nothing is queued when an error is returned.  n == 0 is a
 * no-op.
 * Paper: "Stepping algorithm" (track initializers, used to fill vacant slots
 * at the start of each step iteration); "Asynchronous memory management"
 * (pinned staging, stream-ordered copy). */
ems_status ems_push_primaries(ems_ctx* ctx, const ems_primary* p, uint64_t n);

/* Enqueue `iterations` step iterations (asynchronous; no host wait).  If
 * `out` is non-NULL, synchronizes and returns the counters after them, and
 * returns CAPACITY (counters filled) if the initializer buffer overflowed.
 * Paper: "Stepping algorithm" (a step iteration is a sequence of action
 * kernels over the track array); "Reindexing track slots" (the sort points,
 * ems_options.sort_policy); "Partitioning track data"
 * (ems_options.init_partition); "Reducing load imbalance"
 * (ems_options.max_substeps). */
ems_status ems_step(ems_ctx* ctx, uint32_t iterations, ems_counters* out);

/* Step until no track is alive, queued or pending, or `max_iterations` is
 * reached (then returns STATE).  The host polls device counters through a
 * pinned buffer every `graph_iterations` (or 16) iterations.  Errors:
 * CAPACITY if the initializer buffer overflowed.
 * Paper: "Stepping algorithm" (the host's outer loop of step iterations);
 * "Asynchronous memory management" (termination read from counters copied to
 * pinned memory, no synchronous copy inside the loop). */
ems_status ems_run(ems_ctx* ctx, uint64_t max_iterations, ems_counters* out);

/* Synchronize and read the counters.
 * Paper: "Integration with Perfetto" (counters such as the active and queued
 * tracks of each step iteration). */
ems_status ems_read_counters(ems_ctx* ctx, ems_counters* out);

/* The counters of the snapshot that the last synchronizing call (ems_step
 * with counters, ems_run, ems_read_counters, ems_poll_completed) read, with
 * no device work and no synchronization: a serving loop that has just polled
 * reads its occupancy here instead of synchronizing a second time.
 * Paper: "Integration with Perfetto" (as ems_read_counters). */
ems_status ems_last_counters(ems_ctx* ctx, ems_counters* out);

/* Events whose tracks have all finished since the last poll (serving): an
 * event completes when its last pushed primary and last secondary have
 * retired.  Writes up to `cap` event ids to `events` (completion order) and
 * their count to *n; synchronizes the stream.  Errors: CAPACITY (and *n = 0)
 * once the initializer buffer has overflowed, since secondaries were dropped
 * and completed events may miss energy.
 * Paper: "GPU thread scaling" (events mixed in one track array on one stream;
 * an event ends when all its tracks have ended). */
ems_status ems_poll_completed(ems_ctx* ctx, uint64_t* events, uint32_t cap, uint32_t* n);

/* Energy deposited per slab (n_slabs values) and the ledger of `event`.
 * Paper: "Asynchronous memory management" (scored energy stays on the device
 * and is read back per event, not copied every iteration). */
ems_status ems_read_edep(ems_ctx* ctx, uint64_t event, double* per_slab, uint32_t n_slabs, ems_ledger* ledger);

/* Read all tally rows at once: edep[max_events][n_slabs], ledgers[max_events]
 * (either may be NULL), plus the event id of every row (row_event, may be
 * NULL; unused rows hold UINT64_MAX).
 * Paper: "Asynchronous memory management" (as ems_read_edep). */
ems_status ems_read_all_tallies(ems_ctx* ctx, double* edep, ems_ledger* ledgers, uint64_t* row_event);

/* Free the tally row of a finished event and zero it for reuse.
 * Paper: "GPU thread scaling" (events mixed in one track array: a finished
 * event's row is reused by the next). */
ems_status ems_release_event(ems_ctx* ctx, uint64_t event);

/* Release n events at once (one clearing kernel).  Errors: INVALID_ARG for an
 * unknown or repeated event id (nothing is released then).
 * Paper: "GPU thread scaling" (as ems_release_event). */
ems_status ems_release_events(ems_ctx* ctx, const uint64_t* events, uint64_t n);

/* ---- test hooks ---------------------------------------------------------- */

/* Give `event` a tally row (as ems_push_primaries would) and return it.
 * Paper: no passage (test hook). */
ems_status ems_debug_register_event(ems_ctx* ctx, uint64_t event, uint32_t* row);

/* Overwrite slots [0, n) with `tracks` (rows from ems_debug_register_event,
 * energies >= the cut), mark every other slot vacant and discard queued
 * secondaries.  Errors: STATE, CAPACITY (n > n_slots), INVALID_ARG.
 * Paper: "Stepping algorithm" (track state arrays; test hook for one step of
 * given states). */
ems_status ems_debug_inject(ems_ctx* ctx, const ems_track* tracks, uint64_t n);

/* Run `iterations` step iterations, skipping the slot initialization phase
 * when `no_init` is nonzero (secondaries then stay in the initializer buffer).
 * Paper: "Stepping algorithm" (one step iteration; test hook). */
ems_status ems_debug_iterate(ems_ctx* ctx, uint32_t iterations, int32_t no_init);

/* Read slots [0, n) into `tracks`.
 * Paper: "Stepping algorithm" (track state arrays; test hook). */
ems_status ems_debug_read_tracks(ems_ctx* ctx, ems_track* tracks, uint64_t n);

/* Read the secondary initializer buffer (up to cap entries) as tracks; *n
 * receives the number queued.
 * Paper: "Stepping algorithm" (the buffer of track initializers; test hook). */
ems_status ems_debug_read_secondaries(ems_ctx* ctx, ems_track* out, uint64_t cap, uint64_t* n);

/* Stable sort of n small keys on the device with `policy` (PARTITION: keys
 * < 16; RADIX: keys < 128; other keys are rejected with
 * EMS_ERR_INVALID_ARG), through the same kernels as a sort point of the step
 * loop; perm[i] = index of the i-th smallest key, equal keys in index order.
 * Allocates and frees its own device buffers.
 * Paper: "Reindexing track slots" (sorting the slot indices, not the state). */
ems_status ems_debug_sort(ems_ctx* ctx, const uint8_t* keys, uint64_t n, int32_t policy, uint32_t* perm);

/* Allocation-free variant of ems_debug_sort, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same stable counting sort of n small
 * keys (PARTITION: keys < 16; RADIX: keys < 128) through the same kernels,
 * with `keys` (n bytes) and `perm` (n uint32) in DEVICE memory owned by the
 * caller, enqueued on the context's stream without any host wait, copy,
 * memset or allocation.  perm[i] = index of the i-th smallest key, equal keys
 * in index order; keys at or above the policy's bin count are left out (perm
 * then holds the valid keys' order in its first entries, the rest untouched).
 * The per-tile histograms live in a fixed device array of the library (4 MiB
 * + 512 B per device, held until the process ends); every word a call reads
 * is written by that call first, so nothing is cleared between calls.  Calls
 * that overlap on one GPU (other streams, other contexts, other threads)
 * share that array and race: serialize them.  The context's device must be
 * current.  Errors: INVALID_ARG (null pointer, policy), CAPACITY (n > 2^23),
 * STATE (another device current), DEVICE. */
ems_status ems_sort_keys_noalloc(ems_ctx* ctx, const uint8_t* keys, uint64_t n, int32_t policy, uint32_t* perm);

/* Run-time tuning (the autotuner's knobs; results do not depend on them).
 * block[i] is the block size of kernel role i (role order as returned by
 * ems_profile_read: vacancies, init, pre_step (unused: the along-step
 * kernels run the pre-step), sort, along_neutral,
 * along_charged, along_field, compton, photoelectric, pair, moller, bhabha,
 * bremsstrahlung, drain, interactions, annihilation); 0 keeps
 * ems_options.block_size.  Below tail_threshold live tracks an iteration
 * skips the reordering and runs masked (the device decides per iteration).
 * phase_sort[p] chooses the reordering per sort point p (0: before the
 * along-step kernels, 1: before the interaction kernels) and occupancy
 * bucket: an iteration with n live tracks (n >= tail_threshold) reorders at
 * sort point p when bit floor(log2 n) of phase_sort[p] is set, and runs that
 * point's kernels masked otherwise (all bits set: reorder at every
 * occupancy; none set: that point's kernels are not launched at all).  The
 * sort policy itself (partition, radix, queue) is one per context.
 *
 * Drain (ems_run only; 0 = off): once the latest counter snapshot shows fewer
 * than drain_threshold tracks alive, queued or pending, and no more than the
 * snapshot before it (the tail of the run, not the ramp of a run that starts
 * with few tracks: the first snapshot never starts it; 0xFFFFFFFF drains from
 * the first iteration on), each further
 * iteration fills the vacant slots and then runs one kernel in which every
 * block steps its own tracks in rounds, for up to drain_steps rounds (> 0)
 * of up to 4 steps per track: half of a block's threads own occupied slots
 * and half vacant ones,
 * secondaries go onto the block's stack of 2048 records and threads with a
 * vacant slot take them (the rest go back to the initializer buffer).  It
 * removes the per-iteration launch latency of the last, nearly empty
 * iterations; the physics is the same per-track code.
 *
 * reuse_parent_slot (0/1): a track that ends in a step hands its slot to its
 * first secondary directly, instead of through the initializer buffer and the
 * next iteration's fill (fewer initializer round trips; it mixes charged and
 * neutral tracks in slots that init_partition would keep apart).
 *
 * fuse_interactions (0/1): run the seven interaction kernels (six processes
 * and annihilation at rest) as one launch that walks the combined index range
 * of the interaction actions (each wave holds one action except at range
 * boundaries) instead of seven launches on the library's streams; kernel role
 * "interactions" in the block table.
 *
 * fuse_along (0/1): with a field and one stream, run the photon and field
 * along-steps as one launch (kernel role "along_field" in the block table and
 * the profile): each thread of the resident grid steps its field tracks, then
 * its share of the photon tracks, dealt out first to the waves that had one
 * field round fewer, so the photon steps fill the end of the field launch.
 * Without a field, or with several streams, it has no effect.  On by default
 * (ems_create); the other knobs default to 0 / off.

 * With ems_options.deterministic set, the queue policy and a drain threshold
 * above 0 are rejected (EMS_ERR_INVALID_ARG).
 * Setting the tuning re-captures graphs on the next run.
 * Paper: "Reindexing track slots" (sort policy, tail threshold, phase
 * table); "Partitioning
 * track data" (parent-slot reuse); "Reducing load imbalance" (the drain of the
 * last tracks); "Performance results" (launch shapes). */
typedef struct {
    int32_t sort_policy;
    uint32_t tail_threshold;
    int32_t block[16];
    uint32_t drain_threshold;
    uint32_t drain_steps;
    uint32_t reuse_parent_slot;
    uint32_t fuse_interactions;
    uint32_t phase_sort[2];
    uint32_t fuse_along;
} ems_tuning;
ems_status ems_set_tuning(ems_ctx* ctx, const ems_tuning* t);
ems_status ems_get_tuning(ems_ctx* ctx, ems_tuning* t);

/* Average duration [ms] of each kernel over the iterations launched since the
 * last call, measured with HIP events around every launch on the library's
 * stream when `enable` was set; names are fixed kernel-role strings.
 * Paper: "Integration with Perfetto" (time per action in each step iteration). */
ems_status ems_profile_enable(ems_ctx* ctx, int32_t enable);
ems_status ems_profile_read(ems_ctx* ctx, const char** names, double* total_ms, uint64_t* launches, uint32_t cap,
                            uint32_t* n);

#ifdef __cplusplus
}
#endif
#endif /* EMSTEP_H */
