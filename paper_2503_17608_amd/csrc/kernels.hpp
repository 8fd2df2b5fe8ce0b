// Step-iteration kernels (paper, "Stepping algorithm"): one kernel per
// stepping action over the track state (an array per field, with the fields
// read together on every step in one record per slot).
//
// Every kernel visits its tracks either masked over all slots (the paper's
// default: each kernel runs on all tracks and masks by next action) or through
// an index range of a sorted permutation of slots (paper, "Reindexing track
// slots").  Index ranges live in device memory so that a captured HIP graph
// replays correctly whatever the occupancy.
#pragma once
#include "common.hpp"
#include "physics.hpp"

namespace ems {

// The fields that both the along-steps and the interactions read and write
// for every track they touch -- position, direction, kinetic energy and the
// random-number key -- sit together in one 64-byte record per slot instead
// of arrays of their own: a kernel that reaches a few scattered slots (the
// interactions after the sort, the fill) then brings in one half line per
// track rather than a line of each array.  Record of slot s at
// base + 64 s: x, y, z (double) at 0, 8, 16; key at 24; ux, uy, uz and T
// (precision R) from 32.
constexpr uint32_t kTrackRec = 64;

// One field of the records, indexed by slot like an array.  Single-field
// accesses go through it; the hot paths read and write whole records with
// load_track / store_track (four 16-byte accesses), which the compiler does
// not form from separate field accesses.
template <class T, uint32_t OFF>
struct RecField {
    char* base;   // the record of slot 0 (aligned to the record size)
    __device__ __forceinline__ T& operator[](size_t i) const
    {
        char* rec = static_cast<char*>(__builtin_assume_aligned(base + i * kTrackRec, kTrackRec));
        return *reinterpret_cast<T*>(rec + OFF);
    }
};

template <class R>
struct Dev {
    // track state over n_slots: an array per field, except the RecField
    // members (key, T, x, y, z, ux, uy, uz), which live in the 64-byte records
    uint8_t* type;
    uint8_t* action;
    uint8_t* flags;
    uint8_t* nsearch;
    uint16_t* slab;
    uint32_t* row;
    uint32_t* step;
    RecField<uint64_t, 24> key;
    RecField<R, 32 + 3 * sizeof(R)> T;
    R* nl;
    R* xs;
    double* sphys;
    double* sdone;
    double* htry;
    RecField<double, 0> x;
    RecField<double, 8> y;
    RecField<double, 16> z;
    RecField<R, 32> ux;
    RecField<R, 32 + sizeof(R)> uy;
    RecField<R, 32 + 2 * sizeof(R)> uz;
    uint32_t n_slots;
    // buffers
    Initializer* queue;
    unsigned long long queue_cap;
    Initializer* prims;
    unsigned long long prim_cap;   // pending primaries form a ring of this size
    uint32_t* vac;
    uint32_t* vac_cnt;      // per vacancy block
    uint32_t* init_cnt;     // per init block: charged initializers
    uint32_t* perm;
    uint32_t* lists;        // queue policy: [A_NUM][n_slots] slot lists of the interaction actions
    Counters* ctr;
    // physics / geometry
    Tables<R> tb;
    const double* zp;
    const int32_t* smat;
    int n_slabs;
    double W;
    double B[3];
    int has_field;
    double ecut;
    uint64_t seed;
    const uint64_t* row_event;
    double* edep;           // [n_rep_e][edep_rs] copies of [rows][edep_stride], summed by readers
    Ledger* ledger;         // [n_rep][ledger_rs] (copies of the per-event ledger, summed by readers)
    unsigned long long* part;   // per-block partial counters [kNumW][part_stride] (no global atomics)
    unsigned int part_stride;
    unsigned int* row_state;    // 1 while an event occupies the row and has not been reported complete
    unsigned int* live;     // [n_rep][live_rs]; per row, summed over the copies: primaries pending +
                            // tracks alive or queued
    unsigned int rep_mask;  // n_rep - 1 (n_rep a power of two)
    unsigned int ledger_rs, live_rs;   // rows per copy (padded to 4 KiB pages)
    unsigned long long* done_ring;  // completed events as (generation << 32 | row), capacity rows
    const unsigned int* row_gen;    // registration generation of each row
    unsigned int n_rows;
    int edep_stride;
    unsigned int edep_rep_mask;   // copies of the deposit tallies - 1 (a power of two)
    unsigned long long edep_rs;   // doubles per copy (padded to 4 KiB pages)
    int max_substeps;
    int sorted;             // along-step kernels: 0 masked over all slots, 1 sorted permutation ranges
    int sorted2;            // interaction kernels: 0 masked, 1 sorted ranges, 2 lists filled by the along-step
    unsigned int tail_threshold;  // below this many live tracks an iteration runs masked (no reordering)
    // per occupancy bucket b = floor(log2 live tracks): bit b set when sort
    // point 1 (before the along-steps) / 2 (before the interactions)
    // reorders in an iteration of that bucket, else its kernels run masked
    unsigned int phase_sort1, phase_sort2;
    // masked iterations of the one-launch along-steps walk the slots occupied
    // before the fill (listed by the vacancy pass) and the filled vacancies,
    // not every slot
    int compact_along;
    uint32_t* along_list;   // [n_slots] occupied slots before the fill, in slot order
    int stage_tables;       // copy the tables into LDS at block start
    int reuse_parent;       // a track that ends hands its slot to its first secondary
    int msc;                // multiple-scattering deflection after charged along-steps
    int fill_reserve;       // partitioned fill by per-block reservations (k_init_reserve), no count pass
    // deterministic appends: secondaries staged per position of the
    // interaction order (up to 3 records each), appended in that order
    int det;
    uint8_t* sec_cnt;       // [n_slots] secondaries staged at a position (0 between iterations)
    Initializer* sec_rec;   // [n_slots][3]
    uint32_t* sec_blk;      // per block of kVacBlock positions: secondaries staged
    const double* x0;       // radiation length per material [cm]
    int n_tab;              // table values (n_materials * 8 * 181)
};

// A whole track record, read and written with 16-byte accesses (the hot
// paths read every field of it, a new track writes every field).
template <class R>
struct alignas(16) TrackRec {
    double r[3];
    uint64_t key;
    R u[3];
    R T;
};
static_assert(sizeof(TrackRec<double>) == kTrackRec && sizeof(TrackRec<float>) <= kTrackRec, "track record size");
static_assert(offsetof(TrackRec<double>, key) == 24 && offsetof(TrackRec<double>, u) == 32 &&
                  offsetof(TrackRec<double>, T) == 56 && offsetof(TrackRec<float>, T) == 44,
              "track record layout (the RecField offsets of Dev)");

template <class R>
__device__ __forceinline__ TrackRec<R> load_track(const Dev<R>& d, uint32_t s)
{
    return *reinterpret_cast<const TrackRec<R>*>(d.x.base + (size_t)s * kTrackRec);
}

template <class R>
__device__ __forceinline__ void store_track(const Dev<R>& d, uint32_t s, const TrackRec<R>& tr)
{
    *reinterpret_cast<TrackRec<R>*>(d.x.base + (size_t)s * kTrackRec) = tr;
}

// Tables used by a block: staged into LDS (one copy per block, read by every
// lookup of the block's tracks) or read through the caches.
template <class R>
__device__ __forceinline__ Tables<R> block_tables(const Dev<R>& d, R* lds)
{
    Tables<R> t = d.tb;
    if (d.stage_tables) {
        for (int i = threadIdx.x; i < d.n_tab; i += blockDim.x) lds[i] = d.tb.v[i];
        __syncthreads();
        t.v = lds;
    }
    return t;
}

constexpr int kVacBlock = 1024;   // slots per block of the vacancy and init kernels
constexpr int kSortThreads = 256;
constexpr int kSortTile = 1024;      // slots per sort block
constexpr int kStepMaxBlock = 512;  // block-size bound of the step kernels (lets them keep state in VGPRs)

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t rank_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Per-block partial counters: every block adds its own entry with a plain
// read-modify-write (only that block writes it during a launch), so hot
// kernels issue no same-address global atomics; the snapshot kernel sums the
// entries.  All threads of the block must call (block-uniform control flow).
__device__ __forceinline__ unsigned long long block_sum(unsigned long long v)
{
    __shared__ unsigned long long red[16];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if (lane_id() == 0) red[w] = v;
    __syncthreads();
    unsigned long long t = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < nw; ++i) t += red[i];
    return t;          // valid in thread 0
}

template <class R>
__device__ __forceinline__ void flush_count(const Dev<R>& d, int role, unsigned long long v)
{
    unsigned long long t = block_sum(v);
    if (threadIdx.x == 0 && t) d.part[(size_t)role * d.part_stride + blockIdx.x] += t;
}

// The same for a role that kernels running concurrently on several streams
// share (the pre-steps of the photon and lepton along-steps, the slot reuse
// of the per-process interaction kernels): block b of two such kernels
// writes the same entry, so the update is atomic (one per block and launch).
template <class R>
__device__ __forceinline__ void flush_count_shared(const Dev<R>& d, int role, unsigned long long v)
{
    unsigned long long t = block_sum(v);
    if (threadIdx.x == 0 && t) atomicAdd(&d.part[(size_t)role * d.part_stride + blockIdx.x], t);
}

// Per-event counters (the ledger and the live count) and the deposit tallies
// are kept in several copies, each in pages of its own: a thread adds to the
// copy of its global index.  An event with many tracks in flight would otherwise funnel every
// retirement, secondary and step count of a launch into a few addresses,
// whose device-scope atomics are performed one after another; spread over
// the copies they proceed in parallel.  Readers sum the copies.
__device__ __forceinline__ uint32_t rep_index(uint32_t mask)
{
    return (blockIdx.x * blockDim.x + threadIdx.x) & mask;
}

template <class R>
__device__ __forceinline__ Ledger& ledger_of(const Dev<R>& d, uint32_t row)
{
    return d.ledger[(size_t)rep_index(d.rep_mask) * d.ledger_rs + row];
}

template <class R>
__device__ __forceinline__ unsigned int* live_of(const Dev<R>& d, uint32_t row)
{
    return d.live + (size_t)rep_index(d.rep_mask) * d.live_rs + row;
}

// A retired track leaves its event (no-return atomic); completion is detected
// after the iteration by the row scan.
template <class R>
__device__ __forceinline__ void leave_event(const Dev<R>& d, bool retired, uint32_t row)
{
    if (retired) atomicSub(live_of(d, row), 1u);
}

// Queue policy: append slot s to the list of action `key` (lanes with act set).
// One atomic per distinct key in the wave; lanes keep their order within it.
template <class R>
__device__ __forceinline__ void append_to_list(const Dev<R>& d, bool act, uint32_t key, uint32_t s)
{
    uint64_t pending = __ballot(act);
    while (pending) {
        int leader = __ffsll((unsigned long long)pending) - 1;
        uint32_t lk = __shfl(key, leader, 64);
        bool mine = act && key == lk;
        uint64_t same = __ballot(mine);
        uint32_t base = 0;
        if (lane_id() == leader) base = atomicAdd(&d.ctr->list_cnt[lk], (uint32_t)__popcll(same));
        base = __shfl(base, leader, 64);
        if (mine) d.lists[(size_t)lk * d.n_slots + base + rank_below(same)] = s;
        pending &= ~same;
    }
}

// exclusive prefix of per-block counts: sum of cnt[0, b) with the whole block
__device__ uint32_t block_prefix(const uint32_t* cnt, uint32_t b, uint32_t* scratch)
{
    uint32_t s = 0;
    for (uint32_t i = threadIdx.x; i < b; i += blockDim.x) s += cnt[i];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    int w = threadIdx.x >> 6;
    if (lane_id() == 0) scratch[w] = s;
    __syncthreads();
    uint32_t tot = 0;
    int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) tot += scratch[i];
    __syncthreads();
    return tot;
}

// ---- vacancy compaction (ordered by slot index) ---------------------------------
// Each thread of the two vacancy kernels covers kVacPer consecutive slots
// (one 4-byte load of their type bytes), so a block covers kVacSpan slots and
// the per-block counts that every block of the scatter adds up stay few
// (256 at 2^20 slots, 2048 at 2^23).
constexpr int kVacPer = 4;
constexpr uint32_t kVacSpan = (uint32_t)kVacBlock * kVacPer;

// Vacancy bits of the kVacPer slots from s0 (bit j: slot s0 + j), and how
// many of those slots exist (fewer than kVacPer only at the end of the array).
template <class R>
__device__ __forceinline__ uint32_t vacant_bits(const Dev<R>& d, uint32_t s0, uint32_t& valid)
{
    static_assert(kVacPer == 4, "one 4-byte load per thread");
    uint32_t m = 0;
    if (s0 + kVacPer <= d.n_slots) {
        // s0 is a multiple of 4 and the type array starts 256-byte aligned
        const uint32_t w = *reinterpret_cast<const uint32_t*>(d.type + s0);
        for (int j = 0; j < kVacPer; ++j) m |= (uint32_t)(((w >> (8 * j)) & 0xFFu) == kDead) << j;
        valid = kVacPer;
    } else {
        valid = s0 < d.n_slots ? d.n_slots - s0 : 0u;
        for (uint32_t j = 0; j < valid; ++j) m |= (uint32_t)(d.type[s0 + j] == kDead) << j;
    }
    return m;
}

template <class R>
__global__ void __launch_bounds__(kVacBlock) k_vac_count(Dev<R> d)
{
    const uint32_t s0 = (blockIdx.x * kVacBlock + threadIdx.x) * kVacPer;
    uint32_t valid = 0;
    const uint32_t m = vacant_bits(d, s0, valid);
    const unsigned long long c = block_sum((unsigned long long)__popc(m));
    if (threadIdx.x == 0) d.vac_cnt[blockIdx.x] = (uint32_t)c;
}

// Writes vacant slot indices in slot order; the last block plans the fill:
// initializers are taken from the top of the secondary buffer first (LIFO),
// then from the pending primaries.
//
// With live_out set, the occupied slots are also listed there in slot order
// (n_slots - n_vac of them), for the drain kernel and the listed walk of the
// along-steps.
template <class R>
__global__ void __launch_bounds__(kVacBlock) k_vac_scatter(Dev<R> d, int plan_fill, uint32_t* live_out)
{
    __shared__ uint32_t red[kVacBlock / 64];
    __shared__ uint32_t wcnt[kVacBlock / 64];
    const uint32_t prefix = block_prefix(d.vac_cnt, blockIdx.x, red);
    const uint32_t s0 = (blockIdx.x * kVacBlock + threadIdx.x) * kVacPer;
    uint32_t valid = 0;
    const uint32_t m = vacant_bits(d, s0, valid);
    const uint32_t nv = (uint32_t)__popc(m);
    // vacancies of the block's earlier threads: a wave scan, then the waves
    const int lane = lane_id(), w = threadIdx.x >> 6;
    uint32_t x = nv;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wcnt[w] = x;
    __syncthreads();
    uint32_t before = 0;
    for (int i = 0; i < w; ++i) before += wcnt[i];
    uint32_t off = prefix + before + x - nv;           // vacancies before slot s0
    for (int j = 0; j < kVacPer; ++j)
        if ((m >> j) & 1u) d.vac[off++] = s0 + (uint32_t)j;
    if (live_out) {
        // every slot before s0 exists, so the occupied ones number s0 - vacancies
        uint32_t lo = s0 - (prefix + before + x - nv);
        for (uint32_t j = 0; j < valid; ++j)
            if (!((m >> j) & 1u)) live_out[lo++] = s0 + j;
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        uint32_t blk = 0;
        for (int i = 0; i < kVacBlock / 64; ++i) blk += wcnt[i];
        Counters* c = d.ctr;
        uint32_t n_vac = prefix + blk;
        c->n_vac = n_vac;
        c->n_alive = d.n_slots - n_vac;
        c->iterations += 1;
        unsigned long long q = c->queue_size;
        if (q > d.queue_cap) q = d.queue_cap;     // entries past capacity were dropped (overflow flagged)
        unsigned long long pa = c->prim_end - c->prim_next;
        unsigned long long tq = 0, tp = 0;
        if (plan_fill) {
            tq = q < n_vac ? q : n_vac;
            unsigned long long left = n_vac - tq;
            tp = pa < left ? pa : left;
        }
        c->n_take_q = (uint32_t)tq;
        c->n_take_p = (uint32_t)tp;
        // the partitioned fill sets its charged count (by reservations: from 0)
        c->n_take_lo = d.fill_reserve ? 0u : (uint32_t)(tq + tp);
        c->n_take_hi = 0u;
        c->q_base = q - tq;
        c->p_base = c->prim_next;
        c->queue_size = q - tq;
        c->prim_next += tp;
        c->alive_before = d.n_slots - n_vac;
        c->n_alive += (uint32_t)(tq + tp);
        c->list_cnt[0] = c->n_alive;
        for (int a = 1; a < 16; ++a) c->list_cnt[a] = 0;     // lists are refilled every iteration
        // this iteration's reordering: by sort point, from the occupancy
        // bucket's entry of the phase table and the tail threshold
        unsigned int ph = 0;
        if (c->n_alive > 0 && c->n_alive >= d.tail_threshold) {
            const int b = 31 - __clz((int)c->n_alive);
            if (d.sorted && ((d.phase_sort1 >> b) & 1u)) ph |= 1u;
            if (d.sorted2 && ((d.phase_sort2 >> b) & 1u)) ph |= 2u;
        }
        c->phase_sorted = ph;
    }
}

// ---- deterministic appends --------------------------------------------------------
// The interaction kernels staged each track's secondaries at its position in
// the interaction order; these two kernels append them to the initializer
// buffer in position order, so the buffer, and with it the slots the next
// fill assigns, repeat exactly from run to run (the paper's deterministic
// vacancy fill).  First the secondaries per block of positions; block 0 also
// records the buffer size the appends start from.
template <class R>
__global__ void __launch_bounds__(kVacBlock) k_sec_count(Dev<R> d)
{
    __shared__ uint32_t red[kVacBlock / 64];
    const uint32_t p = blockIdx.x * kVacBlock + threadIdx.x;
    uint32_t c = p < d.n_slots ? d.sec_cnt[p] : 0u;
    for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o, 64);
    if (lane_id() == 0) red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int i = 0; i < kVacBlock / 64; ++i) t += red[i];
        d.sec_blk[blockIdx.x] = t;
        if (blockIdx.x == 0) d.ctr->sec_base = d.ctr->queue_size;
    }
}

// Then each position's records go to sec_base + (secondaries staged at
// earlier positions); the staging counts are cleared for the next iteration
// and the last block sets the buffer size.
template <class R>
__global__ void __launch_bounds__(kVacBlock) k_sec_scatter(Dev<R> d)
{
    __shared__ uint32_t red[kVacBlock / 64];
    __shared__ uint32_t wsum[kVacBlock / 64];
    const uint32_t prefix = block_prefix(d.sec_blk, blockIdx.x, red);
    const uint32_t p = blockIdx.x * kVacBlock + threadIdx.x;
    const uint32_t c = p < d.n_slots ? d.sec_cnt[p] : 0u;
    const int lane = lane_id(), w = threadIdx.x >> 6;
    uint32_t x = c;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    uint32_t off = prefix + (x - c);
    for (int i = 0; i < w; ++i) off += wsum[i];
    const unsigned long long base = d.ctr->sec_base;
    for (uint32_t k = 0; k < c; ++k) {
        const unsigned long long q = base + off + k;
        if (q < d.queue_cap) d.queue[q] = d.sec_rec[(size_t)p * 3 + k];
        else atomicOr(&d.ctr->overflow, 1u);
    }
    if (c) d.sec_cnt[p] = 0;
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        uint32_t blk = 0;
        for (int i = 0; i < kVacBlock / 64; ++i) blk += wsum[i];
        d.ctr->queue_size = base + prefix + blk;
    }
}

template <class R>
__device__ __forceinline__ const Initializer* taken(const Dev<R>& d, uint32_t i)
{
    const Counters* c = d.ctr;
    if (i < c->n_take_q) return &d.queue[c->q_base + c->n_take_q - 1 - i];
    return &d.prims[(c->p_base + (i - c->n_take_q)) % d.prim_cap];
}

// A new track in `slot` from an initializer record.
template <class R>
__device__ __forceinline__ void init_slot(const Dev<R>& d, uint32_t slot, const Initializer& rec)
{
    // the path length, search state, step limit and cross section of a
    // step are read only when it resumes from a pause: a new track has none
    d.type[slot] = rec.type;
    d.action[slot] = A_IDLE;
    d.flags[slot] = 0;
    d.slab[slot] = rec.slab;
    d.row[slot] = rec.row;
    d.step[slot] = 0;
    d.nl[slot] = R(-1);
    TrackRec<R> tr;
    tr.r[0] = rec.r[0];
    tr.r[1] = rec.r[1];
    tr.r[2] = rec.r[2];
    tr.key = rec.key;
    tr.u[0] = (R)rec.u[0];
    tr.u[1] = (R)rec.u[1];
    tr.u[2] = (R)rec.u[2];
    tr.T = (R)rec.T;
    store_track(d, slot, tr);
}

// per-block count of charged initializers among the taken ones (partitioned fill)
template <class R>
__global__ void __launch_bounds__(kVacBlock) k_init_count(Dev<R> d)
{
    uint32_t i = blockIdx.x * kVacBlock + threadIdx.x;
    uint32_t n = d.ctr->n_take_q + d.ctr->n_take_p;
    int ch = 0;
    if (i < n) ch = taken(d, i)->type != kGamma;
    int c = __syncthreads_count(ch);
    if (threadIdx.x == 0) d.init_cnt[blockIdx.x] = (uint32_t)c;
}

// Fill vacancies from the taken initializers.  Without partitioning the i-th
// taken initializer goes to the i-th vacancy; with it, charged initializers
// fill vacancies from the lowest slot upwards and neutral ones from the
// highest slot downwards (paper, "Partitioning track data").
template <class R, bool PART>
__global__ void __launch_bounds__(kVacBlock) k_init(Dev<R> d)
{
    __shared__ uint32_t red[kVacBlock / 64];
    __shared__ uint32_t wcnt[kVacBlock / 64];
    const Counters* c = d.ctr;
    uint32_t n = c->n_take_q + c->n_take_p;
    if (blockIdx.x * kVacBlock >= n) return;          // block-uniform
    uint32_t i = blockIdx.x * kVacBlock + threadIdx.x;
    bool act = i < n;
    Initializer rec;
    if (act) rec = *taken(d, i);
    uint32_t slot = 0;
    if (PART) {
        uint32_t prefix = block_prefix(d.init_cnt, blockIdx.x, red);
        bool ch = act && rec.type != kGamma;
        uint64_t m = __ballot(ch);
        int w = threadIdx.x >> 6;
        if (lane_id() == 0) wcnt[w] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t off = prefix;
        for (int k = 0; k < w; ++k) off += wcnt[k];
        uint32_t cidx = off + rank_below(m);          // charged initializers before i
        if (act) slot = ch ? d.vac[cidx] : d.vac[c->n_vac - 1 - (i - cidx)];
        // the last block knows how many charged initializers there are
        if (threadIdx.x == 0 && (blockIdx.x + 1) * kVacBlock >= n) {
            uint32_t tot = prefix;
            for (int k = 0; k < kVacBlock / 64; ++k) tot += wcnt[k];
            d.ctr->n_take_lo = tot;
        }
    } else {
        if (act) slot = d.vac[i];
    }
    flush_count(d, W_INIT, act ? 1ull : 0ull);
    if (!act) return;
    init_slot(d, slot, rec);
}

// Partitioned fill without a count pass: each block reserves room for its
// charged initializers from the low end of the vacancies and for its neutral
// ones from the high end with one atomic each, then places them in lane
// order.  The set of slots filled is the one k_init<R, true> fills; which
// charged initializer lands in which of them follows the order in which the
// blocks reserve (the physics does not depend on it: random numbers are
// keyed by track).  n_take_lo ends as the number of charged initializers.
template <class R>
__global__ void __launch_bounds__(kVacBlock) k_init_reserve(Dev<R> d)
{
    __shared__ uint32_t wch[kVacBlock / 64], wne[kVacBlock / 64];
    __shared__ uint32_t base_lo, base_hi;
    Counters* c = d.ctr;
    const uint32_t n = c->n_take_q + c->n_take_p;
    if (blockIdx.x * kVacBlock >= n) return;          // block-uniform
    const uint32_t i = blockIdx.x * kVacBlock + threadIdx.x;
    const bool act = i < n;
    Initializer rec;
    if (act) rec = *taken(d, i);
    const bool ch = act && rec.type != kGamma, ne = act && !ch;
    const uint64_t mc = __ballot(ch), mn = __ballot(ne);
    const int w = threadIdx.x >> 6;
    if (lane_id() == 0) {
        wch[w] = (uint32_t)__popcll(mc);
        wne[w] = (uint32_t)__popcll(mn);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tc = 0, tn = 0;
        for (int k = 0; k < kVacBlock / 64; ++k) {
            tc += wch[k];
            tn += wne[k];
        }
        base_lo = tc ? atomicAdd(&c->n_take_lo, tc) : 0u;
        base_hi = tn ? atomicAdd(&c->n_take_hi, tn) : 0u;
    }
    __syncthreads();
    uint32_t oc = base_lo, on = base_hi;
    for (int k = 0; k < w; ++k) {
        oc += wch[k];
        on += wne[k];
    }
    uint32_t slot = 0;
    if (ch) slot = d.vac[oc + rank_below(mc)];
    if (ne) slot = d.vac[c->n_vac - 1 - (on + rank_below(mn))];
    flush_count(d, W_INIT, act ? 1ull : 0ull);
    if (!act) return;
    init_slot(d, slot, rec);
}

// The along-step action a live slot takes this iteration, from its type alone
// (a paused field step resumes as a field step): the key of the first sort,
// known before the pre-step, which the along-step kernels run themselves.
template <class R>
__device__ __forceinline__ uint8_t along_action(const Dev<R>& d, uint32_t s)
{
    const uint8_t t = d.type[s];
    if (t == kDead) return A_NONE;
    if (t == kGamma) return A_NEUTRAL;
    if (!d.has_field) return A_CHARGED;
    return A_FIELD;
}

// ---- work distribution ----------------------------------------------------------
// Iterate the tracks of action `a`: masked over all slots, or the index range
// of `a` in the sorted permutation (or its list), which holds exactly the
// tracks of that action, so only the masked walk checks the action byte.  The
// loop bound is block-uniform so every wave reaches the converged point at the
// end of each trip.
#define EMS_TRACK_RANGE(d, a)                                                              \
    unsigned long long _work = 0;                                                           \
    const int _mode = (a) >= A_PROC0 ? (((d).ctr->phase_sorted & 2u) ? (d).sorted2 : 0)           \
                                     : (((d).ctr->phase_sorted & 1u) ? (d).sorted : 0);            \
    const uint32_t _n = _mode == 2 ? (d).ctr->list_cnt[a]                                    \
                        : (_mode ? (d).ctr->range_cnt[a] : (d).n_slots);                     \
    const uint32_t _off = _mode == 1 ? (d).ctr->range_off[a] : 0u;                          \
    if (blockIdx.x * blockDim.x >= _n) return;

#define EMS_FOR_TRACKS(d, a, s, act, role)                                                 \
    for (uint32_t _base = blockIdx.x * blockDim.x; _base < _n; _base += gridDim.x * blockDim.x) { \
        uint32_t _i = _base + threadIdx.x;                                                  \
        bool act = _i < _n;                                                                 \
        uint32_t s = 0;                                                                     \
        if (act) s = _mode == 2 ? (d).lists[(size_t)(a) * (d).n_slots + _i]                 \
                     : (_mode ? (d).perm[_off + _i] : _i);                                  \
        if (act && _mode == 0 && ((a) < A_PROC0 ? along_action((d), s) : (d).action[s]) != (a)) \
            act = false;                                                                    \
        _work += act ? 1u : 0u;

#define EMS_END_TRACKS }

// ---- secondary append (block-aggregated) ------------------------------------------
// One global atomic per block that has secondaries (none if it has none);
// lanes get consecutive initializer records in lane order within each wave.
// The event's counters change once per thread: one atomic per secondary
// type created, and one on the live count for the secondaries pushed minus
// the track itself when it ends in this step (`retiring`), none when they
// cancel.  All threads of the block must call it (block-uniform control
// flow).
template <class R>
__device__ __forceinline__ Initializer secondary_record(const Sec<R>& v, const double r[3], uint32_t row,
                                                       uint16_t slab)
{
    Initializer rec;
    rec.T = (double)v.T;
    rec.r[0] = r[0]; rec.r[1] = r[1]; rec.r[2] = r[2];
    rec.u[0] = (double)v.ux; rec.u[1] = (double)v.uy; rec.u[2] = (double)v.uz;
    rec.key = v.key;
    rec.row = row;
    rec.slab = slab;
    rec.type = (uint8_t)v.type;
    rec.pad = 0;
    return rec;
}

// The event's counters for the secondaries of one track (and the track
// itself when it ends in this step).
template <class R>
__device__ __forceinline__ void count_secondaries(const Dev<R>& d, uint32_t row, unsigned int n_gam,
                                                  unsigned int n_ele, unsigned int n_pos, bool retiring)
{
    if (n_gam) atomicAdd(&ledger_of(d, row).n_sec[kGamma], (unsigned long long)n_gam);
    if (n_ele) atomicAdd(&ledger_of(d, row).n_sec[kElectron], (unsigned long long)n_ele);
    if (n_pos) atomicAdd(&ledger_of(d, row).n_sec[kPositron], (unsigned long long)n_pos);
    const int dlive = (int)(n_gam + n_ele + n_pos) - (retiring ? 1 : 0);
    if (dlive != 0) atomicAdd(live_of(d, row), (unsigned int)dlive);    // modulo 2^32: a decrement for -1
}

// `at` is the track's position in the interaction order of this iteration
// (its index in the sort permutation, or its slot when unsorted): with
// deterministic appends the secondaries are staged there and appended in
// position order after the interaction kernels (k_sec_count,
// k_sec_scatter); otherwise they go straight to the buffer, in an order that
// depends on which blocks run first.  (DET is a template parameter so that
// the default kernels compile without the staging path.)
template <class R, bool DET>
__device__ __forceinline__ void append_secondaries(const Dev<R>& d, const SecBuf<R>& sb, uint32_t row,
                                                   uint16_t slab, const double r[3], bool retiring, uint32_t at)
{
    __shared__ unsigned int wtot[16];
    __shared__ unsigned long long bbase;
    const int n = sb.n;
    if (DET) {
        unsigned int n_gam = 0, n_ele = 0, n_pos = 0;
        sb.each([&](const Sec<R>& v, int k) {
            d.sec_rec[(size_t)at * 3 + k] = secondary_record(v, r, row, slab);
            n_gam += v.type == kGamma;
            n_ele += v.type == kElectron;
            n_pos += v.type == kPositron;
        });
        if (n) d.sec_cnt[at] = (uint8_t)n;
        count_secondaries(d, row, n_gam, n_ele, n_pos, retiring);
        return;
    }
    if (__syncthreads_count(n) == 0) {           // block-uniform
        if (retiring) atomicSub(live_of(d, row), 1u);
        return;
    }
    const int lane = lane_id(), w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    int x = n;
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wtot[w] = (unsigned int)x;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned int tot = 0;
        for (int i = 0; i < nw; ++i) {
            unsigned int t = wtot[i];
            wtot[i] = tot;                            // exclusive prefix per wave
            tot += t;
        }
        bbase = atomicAdd(&d.ctr->queue_size, (unsigned long long)tot);
    }
    __syncthreads();
    unsigned long long pos = bbase + wtot[w] + (unsigned long long)(x - n);
    unsigned int n_gam = 0, n_ele = 0, n_pos = 0;
    sb.each([&](const Sec<R>& v, int k) {
        unsigned long long q = pos + (unsigned long long)k;
        if (q >= d.queue_cap) {
            atomicOr(&d.ctr->overflow, 1u);
            return;
        }
        d.queue[q] = secondary_record(v, r, row, slab);
        n_gam += v.type == kGamma;
        n_ele += v.type == kElectron;
        n_pos += v.type == kPositron;
    });
    count_secondaries(d, row, n_gam, n_ele, n_pos, retiring);
    __syncthreads();                                  // wtot / bbase are reused by the next trip
}

template <class R>
__device__ __forceinline__ void record_tally(const Dev<R>& d, uint32_t row, int slab, const StepTally& tl)
{
    if (tl.edep != 0.0)
        atomicAdd(&d.edep[(size_t)rep_index(d.edep_rep_mask) * d.edep_rs + (size_t)row * d.edep_stride + slab],
                  tl.edep);
    if (tl.n_pair) atomicAdd(&ledger_of(d, row).n_pair, (unsigned long long)tl.n_pair);
    if (tl.n_annih) atomicAdd(&ledger_of(d, row).n_annih, (unsigned long long)tl.n_annih);
    if (tl.capped) atomicAdd(&ledger_of(d, row).n_reject_cap, 1ull);
}

// a track finishes: free its slot and add its steps to the event ledger (the
// global step counter is summed per wavefront by the caller)
template <class R>
__device__ __forceinline__ void retire(const Dev<R>& d, uint32_t s, uint32_t row, uint32_t steps)
{
    d.type[s] = kDead;
    d.action[s] = A_NONE;
    atomicAdd(&ledger_of(d, row).steps, (unsigned long long)steps);
}

// Parent-slot reuse: a track that ended in this step hands its slot to its
// first secondary, which then skips the initializer buffer and the fill of
// the next iteration.  The secondary is a new track in every other respect
// (step 0, interaction length unset).  Returns 1 when the slot was reused.
template <class R>
__device__ __forceinline__ uint32_t reuse_slot(const Dev<R>& d, uint32_t s, SecBuf<R>& sb, uint32_t row,
                                               uint16_t slab, const double r[3])
{
    if (!d.reuse_parent || sb.n == 0) return 0u;
    const Sec<R> v = sb.s0;
    Initializer rec;
    rec.T = (double)v.T;
    rec.r[0] = r[0]; rec.r[1] = r[1]; rec.r[2] = r[2];
    rec.u[0] = (double)v.ux; rec.u[1] = (double)v.uy; rec.u[2] = (double)v.uz;
    rec.key = v.key;
    rec.row = row;
    rec.slab = slab;
    rec.type = (uint8_t)v.type;
    rec.pad = 0;
    init_slot(d, s, rec);
    atomicAdd(&ledger_of(d, row).n_sec[v.type], 1ull);
    atomicAdd(live_of(d, row), 1u);
    sb.s0 = sb.s1;
    sb.s1 = sb.s2;
    sb.n -= 1;
    return 1u;
}

// Pre-step of one live, non-paused track, in registers (the caller loaded
// its fields once and stores what persists once): draws the interaction
// length when it is unset, and gives the total cross section, the physics
// step limit, the step's flags (F_DREW, F_LOSS; a new step starts with no
// other flag) and the random word of the step's process selection.  The along-step kernels and the drain run it for their tracks
// before the step; there is no separate pre-step launch.
template <class R>
__device__ __forceinline__ void pre_step(const Dev<R>& d, const Tables<R>& tb, int mat, int typ, R T, R& nl,
                                         uint64_t event, uint64_t key, uint32_t step, R& sig, double& s_phys,
                                         uint8_t& nf, uint64_t& w_sel)
{
    // Block 0 of the step's uniforms, computed once: word 0 is the
    // interaction-length uniform when one is drawn, and the next unused word
    // is the process-selection uniform of the step's end (`w_sel`).  A wave
    // evaluates the block for all its lanes whenever any of them draws, so
    // keeping the word spares the end of the step a second evaluation.
    const U64x4 b0 = philox4x64_10(key, (uint64_t)step, 0, 0, d.seed, event);
    nf = 0;
    w_sel = b0.w[0];
    if (nl < R(0)) {
        nl = -m_log(unit_from<R>(b0.w[0]));
        nf |= F_DREW;
        w_sel = b0.w[1];
    }
    Loc<R> l = locate(tb, T);
    sig = total_xs(tb, mat, typ, T, l, R(d.ecut));
    R s_int = sig > R(0) ? nl / sig : R(INFINITY);
    R sp = s_int;
    if (typ != kGamma) {
        R Rg = interp(range_tab(tb, mat, typ), l);
        R s_loss = Rg <= R(kRFinal) ? Rg : m_max(R(kRFinal), R(kRhoRange) * Rg);
        if (s_loss < s_int) {
            sp = s_loss;
            nf |= F_LOSS;
        }
    }
    s_phys = (double)sp;
}

// ---- pre-step: interaction length, physics step limit, along-step action -----------
// ---- geometry helpers -----------------------------------------------------------
__device__ __forceinline__ double face_plane(const double* zp, int slab, double W, int face)
{
    switch (face) {
    case F_ZLO: return zp[slab];
    case F_ZHI: return zp[slab + 1];
    case F_XLO: return -W;
    case F_XHI: return W;
    case F_YLO: return -W;
    default:    return W;
    }
}
__device__ __forceinline__ int face_axis(int face) { return face <= F_ZHI ? 2 : (face <= F_XHI ? 0 : 1); }

// straight-line distance to leave the slab box (z face wins ties, then x, y)
__device__ __forceinline__ double straight_distance(const double r[3], const double u[3], double zlo, double zhi,
                                                    double W, int* face)
{
    double dz = INFINITY, dx = INFINITY, dy = INFINITY;
    int fz = F_NONE, fx = F_NONE, fy = F_NONE;
    if (u[2] > 0.0) { dz = (zhi - r[2]) / u[2]; fz = F_ZHI; }
    else if (u[2] < 0.0) { dz = (zlo - r[2]) / u[2]; fz = F_ZLO; }
    if (u[0] > 0.0) { dx = (W - r[0]) / u[0]; fx = F_XHI; }
    else if (u[0] < 0.0) { dx = (-W - r[0]) / u[0]; fx = F_XLO; }
    if (u[1] > 0.0) { dy = (W - r[1]) / u[1]; fy = F_YHI; }
    else if (u[1] < 0.0) { dy = (-W - r[1]) / u[1]; fy = F_YLO; }
    dz = fmax(dz, 0.0); dx = fmax(dx, 0.0); dy = fmax(dy, 0.0);
    double dd = dz;
    *face = fz;
    if (dx < dd) { dd = dx; *face = fx; }
    if (dy < dd) { dd = dy; *face = fy; }
    return dd;
}

// Multiple scattering (optional): a charged track still in the stack after
// its along-step of length s is deflected by a space angle theta0 sqrt(-2 ln
// U_a), azimuth 2 pi U_b, where theta0 is the Highland width of the
// projected angle (PDG review, multiple scattering through small angles),
//     theta0 = 13.6 MeV / (beta c p) sqrt(x) (1 + 0.038 ln(x / beta^2)),
// x = s / X0, at the pre-step energy; no deflection for s = 0 or a
// non-positive bracket.  U_a, U_b: words 0 and 1 of the Philox block at
// counter (key, step, 0, 5).  Computed in FP64 in both precisions.
__device__ __forceinline__ void msc_deflect(uint64_t seed, uint64_t event, uint64_t key, uint32_t step, double T_pre,
                                            double s, double X0, double u[3])
{
    if (!(s > 0.0)) return;
    const double p = sqrt(T_pre * (T_pre + 2.0 * kMe));
    const double beta = p / (T_pre + kMe);
    const double x = s / X0;
    const double bracket = 1.0 + 0.038 * log(x / (beta * beta));
    if (!(bracket > 0.0)) return;
    const double theta0 = 13.6 / (beta * p) * sqrt(x) * bracket;
    const U64x4 w = philox4x64_10(key, (uint64_t)step, 0, 5, seed, event);
    const double theta = theta0 * sqrt(-2.0 * log(unit_from<double>(w.w[0])));
    double sp, cp;
    sincos(2.0 * kPi * unit_from<double>(w.w[1]), &sp, &cp);
    double out[3];
    rotate<double>(u, cos(theta), sp, cp, out);
    normalize3<double>(out);
    u[0] = out[0]; u[1] = out[1]; u[2] = out[2];
}

// A lepton stops in its along-step: its kinetic energy is deposited in the
// step's slab.  A positron annihilates at rest; when its photons are below the
// production cut their energy is deposited here as well, otherwise the
// positron keeps its slot and returns true: the interaction launch of this
// iteration creates the photons (with the stopping step's index, so with the
// same random numbers), and the along-step itself creates no tracks.
template <class R>
__device__ __forceinline__ bool stop_defers(const Dev<R>& d, int typ, R& T, StepTally& tl)
{
    tl.edep += (double)T;
    T = R(0);
    if (typ != kPositron) return false;
    if (kMe >= d.ecut) return true;
    tl.n_annih += 1;
    tl.edep += 2.0 * kMe;
    return false;
}

// Common end of an along-step (S6-S8) for a step of length step_len: energy
// loss, the stop, boundary crossing or escape, the choice of the discrete
// process, the step guard.  Clears `alive` when the track ends and sets the
// next action; a positron that stops stays alive with A_ANNIH (annihilation
// at rest, done by the interaction launch), so no along-step creates tracks.
template <class R, bool CHARGED>
__device__ __forceinline__ void finish_along(const Dev<R>& d, const Tables<R>& tb, int typ, R& T, R sig, double step_len,
                                             int face, uint8_t& fl, int mat, uint16_t& slab, StepTally& tl,
                                             bool& alive, uint8_t& next_action, R& nl, uint32_t& step, uint64_t key,
                                             uint64_t event, uint32_t row, bool have_sel, uint64_t w_sel)
{
    // step, key and row come in registers (loaded with the rest of the
    // track up front); step leaves as the track's step count after this step
    const uint32_t k = step;
    if (CHARGED) {
        const R* Rt = range_tab(tb, mat, typ);
        Loc<R> l = locate(tb, T);
        R Rg = interp(Rt, l);
        bool stop = false;
        if (face == F_NONE && (fl & F_LOSS) && Rg <= R(kRFinal)) {
            stop = true;
        } else {
            R Tn = inverse_range(tb, Rt, (R)((double)Rg - step_len), l.i + 1);
            if (Tn < R(d.ecut)) stop = true;
            else {
                tl.edep += (double)T - (double)Tn;
                T = Tn;
            }
        }
        if (stop) {
            if (stop_defers(d, typ, T, tl)) {
                next_action = A_ANNIH;
            } else {
                alive = false;
                next_action = A_NONE;
                step = k + 1;
            }
            return;
        }
    }
    nl = nl - (R)step_len * sig;
    if (face != F_NONE) {
        int next = slab;
        if (face == F_ZLO) next = slab - 1;
        else if (face == F_ZHI) next = slab + 1;
        else next = -1;
        if (next < 0 || next >= d.n_slabs) {
            atomicAdd(&ledger_of(d, row).escaped, (double)T);
            alive = false;
            next_action = A_NONE;
        } else {
            slab = (uint16_t)next;
            next_action = A_IDLE;
        }
        step = k + 1;
    } else if (fl & F_LOSS) {
        next_action = A_IDLE;
        step = k + 1;
    } else {
        // the process-selection uniform: kept from the pre-step's block, or
        // (a step resumed after a pause, which ran no pre-step) drawn here
        R U1;
        if (have_sel) {
            U1 = unit_from<R>(w_sel);
        } else {
            StepRng<R> rng(d.seed, event, key, k, (fl & F_DREW) ? 1 : 0);
            U1 = rng.next();
        }
        R sig1;
        Loc<R> l1;
        l1 = locate(tb, T);
        if (CHARGED) sig1 = total_xs(tb, mat, typ, T, l1, R(d.ecut));
        else sig1 = sig;
        nl = R(-1);
        if (sig1 > R(0)) {
            R target = U1 * sig1, cum = R(0);
            int proc = proc_of(typ, n_proc(typ) - 1);
            for (int k = 0; k < n_proc(typ); ++k) {
                cum += proc_xs(tb, mat, proc_of(typ, k), T, l1, R(d.ecut));
                if (target < cum) { proc = proc_of(typ, k); break; }
            }
            next_action = (uint8_t)(A_PROC0 + proc);
        } else {
            next_action = A_IDLE;
            step = k + 1;
        }
    }
    if (alive && step > kMaxSteps && next_action == A_IDLE) {
        // step guard: the track stops after this (counted) step; a positron
        // annihilates at rest with the counted step's index
        atomicAdd(&ledger_of(d, row).n_guard, 1ull);
        if (typ == kGamma) {
            tl.edep += (double)T;
            T = R(0);
            alive = false;
            next_action = A_NONE;
        } else if (stop_defers(d, typ, T, tl)) {
            next_action = A_ANNIH;
            fl = (uint8_t)((fl & (uint8_t)~F_PAUSED) | F_COUNTED);
        } else {
            alive = false;
            next_action = A_NONE;
        }
    }
}

// Along-step of one straight-line track (photon, or charged without field),
// its pre-step first: the track's fields are loaded once, the step runs in
// registers and what persists goes back to the slot once; the step's deposit
// goes to its tally row.  `row` is the track's row, `next` the next action,
// `retired` the steps of a track that finished (0 while it lives).
template <class R, bool CHARGED>
__device__ __forceinline__ void along_straight_track(const Dev<R>& d, const Tables<R>& tb, uint32_t s, uint32_t& row,
                                                     uint8_t& next, uint32_t& retired)
{
    const int typ = d.type[s];
    row = d.row[s];
    uint16_t slab = d.slab[s];
    const uint16_t slab0 = slab;
    const TrackRec<R> tr = load_track(d, s);
    R T = tr.T;
    R u[3] = {tr.u[0], tr.u[1], tr.u[2]};
    double r[3] = {tr.r[0], tr.r[1], tr.r[2]};
    R nl = d.nl[s];
    uint32_t step = d.step[s];
    const uint64_t key = tr.key;
    const uint64_t event = d.row_event[row];
    const int mat = d.smat[slab];
    R sig;
    double s_phys;
    uint8_t fl;
    uint64_t w_sel;
    pre_step(d, tb, mat, typ, T, nl, event, key, step, sig, s_phys, fl, w_sel);
    double ud[3] = {(double)u[0], (double)u[1], (double)u[2]};
    int face;
    double s_geo = straight_distance(r, ud, d.zp[slab], d.zp[slab + 1], d.W, &face);
    double st;
    if (s_geo <= s_phys) st = s_geo;
    else { st = s_phys; face = F_NONE; }
    r[0] = r[0] + st * ud[0];
    r[1] = r[1] + st * ud[1];
    r[2] = r[2] + st * ud[2];
    if (face != F_NONE) r[face_axis(face)] = face_plane(d.zp, slab, d.W, face);
    StepTally tl = {0.0, 0, 0, 0};
    bool alive = true;
    uint8_t na = A_IDLE;
    const uint32_t k0 = step;
    const double T_pre = (double)T;
    finish_along<R, CHARGED>(d, tb, typ, T, sig, st, face, fl, mat, slab, tl, alive, na, nl, step, key, event, row,
                             true, w_sel);
    record_tally(d, row, slab0, tl);
    if (alive) {
        // the whole record is written (whole 32-byte sectors, no partial
        // writes), the direction unchanged unless deflected
        TrackRec<R> out;
        out.r[0] = r[0];
        out.r[1] = r[1];
        out.r[2] = r[2];
        out.key = key;
        out.u[0] = u[0];
        out.u[1] = u[1];
        out.u[2] = u[2];
        if (CHARGED && d.msc && na != A_ANNIH) {
            msc_deflect(d.seed, event, key, k0, T_pre, st, d.x0[mat], ud);
            out.u[0] = (R)ud[0];
            out.u[1] = (R)ud[1];
            out.u[2] = (R)ud[2];
        }
        out.T = T;
        store_track(d, s, out);
        d.nl[s] = nl;
        if (slab != slab0) d.slab[s] = slab;
        if (step != k0) d.step[s] = step;
        d.flags[s] = fl;
        d.action[s] = na;
        next = na;
    } else {
        retired = step;
        retire(d, s, row, retired);
    }
}

// ---- along-step, straight line (photons, or charged without field) ------------------
template <class R, bool CHARGED>
__global__ void __launch_bounds__(kStepMaxBlock) k_along_straight(Dev<R> d)
{
    extern __shared__ __align__(16) unsigned char ems_lds[];
    const uint8_t A = CHARGED ? A_CHARGED : A_NEUTRAL;
    EMS_TRACK_RANGE(d, A)
    const Tables<R> tb = block_tables(d, (R*)ems_lds);
    unsigned long long ret_acc = 0, pre_acc = 0;
    EMS_FOR_TRACKS(d, A, s, act, CHARGED ? W_CHARGED : W_NEUTRAL)
    uint32_t row = 0;
    uint8_t next = A_NONE;
    uint32_t retired = 0;
    if (act) {
        ++pre_acc;
        along_straight_track<R, CHARGED>(d, tb, s, row, next, retired);
    }
    leave_event(d, retired != 0, row);
    ret_acc += retired;
    if (d.sorted2 == 2 && (d.ctr->phase_sorted & 2u)) append_to_list(d, next >= A_PROC0 && next < A_NUM, next, s);
    EMS_END_TRACKS
    flush_count(d, CHARGED ? W_CHARGED : W_NEUTRAL, _work);
    flush_count(d, kStepsSlot + (CHARGED ? W_CHARGED : W_NEUTRAL), ret_acc);
    flush_count_shared(d, W_PRE, pre_acc);
}

// ---- along-step in a uniform field -------------------------------------------------
__device__ __forceinline__ void rk4(const double r[3], const double u[3], double h, double kf, const double B[3],
                                    double r1[3], double u1[3])
{
    double k1[3], k2[3], k3[3], k4[3], u2[3], u3[3], u4[3];
#define EMS_CROSS(a, o)                                 \
    o[0] = kf * (a[1] * B[2] - a[2] * B[1]);            \
    o[1] = kf * (a[2] * B[0] - a[0] * B[2]);            \
    o[2] = kf * (a[0] * B[1] - a[1] * B[0]);
    EMS_CROSS(u, k1)
    for (int c = 0; c < 3; ++c) u2[c] = u[c] + 0.5 * h * k1[c];
    EMS_CROSS(u2, k2)
    for (int c = 0; c < 3; ++c) u3[c] = u[c] + 0.5 * h * k2[c];
    EMS_CROSS(u3, k3)
    for (int c = 0; c < 3; ++c) u4[c] = u[c] + h * k3[c];
    EMS_CROSS(u4, k4)
#undef EMS_CROSS
    for (int c = 0; c < 3; ++c) {
        r1[c] = r[c] + h / 6.0 * (u[c] + 2.0 * u2[c] + 2.0 * u3[c] + u4[c]);
        u1[c] = u[c] + h / 6.0 * (k1[c] + 2.0 * k2[c] + 2.0 * k3[c] + k4[c]);
    }
}

__device__ __forceinline__ bool beyond(int face, double v, double p)
{
    return (face == F_ZLO || face == F_XLO || face == F_YLO) ? (v < p) : (v > p);
}

__device__ __forceinline__ bool points_out(const double u[3], int face)
{
    switch (face) {
    case F_ZLO: return u[2] < 0.0;
    case F_ZHI: return u[2] > 0.0;
    case F_XLO: return u[0] < 0.0;
    case F_XHI: return u[0] > 0.0;
    case F_YLO: return u[1] < 0.0;
    default:    return u[1] > 0.0;
    }
}

template <class R>
__device__ __forceinline__ void store_dir(double u[3])
{
    // directions are stored in precision R; keep the integrator's copy
    // identical to what a paused step would store
    u[0] = (double)(R)u[0];
    u[1] = (double)(R)u[1];
    u[2] = (double)(R)u[2];
}

__device__ __forceinline__ void normalize_d(double v[3])
{
    double n = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    v[0] /= n; v[1] /= n; v[2] /= n;
}

// Along-step of one charged track in the uniform field, its pre-step first
// unless the step resumes from a pause, with at most `max_sub` RK4
// evaluations (0: no cap) before the step pauses.  The track's fields are
// loaded once; the path length, search state, step limit and cross section
// of a step live in registers and go to the slot only when the step pauses.
// Outputs as for the straight-line step, plus the RK4 evaluations made
// (`att`), whether the step paused (`paused_n`) and whether the pre-step ran
// (`pre_n`).
// The fields a field step reads first, loaded together (the field kernel
// loads the next track's while it steps the current one).
template <class R>
struct FieldIn {
    uint8_t typ, fl;
    uint16_t slab;
    uint32_t row, step;
    uint64_t key;
    R T, nl;
    R u[3];
    double r[3];
};

template <class R>
__device__ __forceinline__ void load_field_in(const Dev<R>& d, uint32_t s, FieldIn<R>& f)
{
    f.typ = d.type[s];
    f.fl = d.flags[s];
    f.slab = d.slab[s];
    f.row = d.row[s];
    f.step = d.step[s];
    const TrackRec<R> tr = load_track(d, s);
    f.key = tr.key;
    f.T = tr.T;
    f.nl = d.nl[s];
    f.u[0] = tr.u[0]; f.u[1] = tr.u[1]; f.u[2] = tr.u[2];
    f.r[0] = tr.r[0]; f.r[1] = tr.r[1]; f.r[2] = tr.r[2];
}

template <class R>
__device__ __forceinline__ void along_field_track(const Dev<R>& d, const Tables<R>& tb, uint32_t s,
                                                  const FieldIn<R>& in, int max_sub, uint32_t& row, uint8_t& next,
                                                  uint32_t& retired, uint32_t& att, uint32_t& paused_n,
                                                  uint32_t& pre_n)
{
    const int typ = in.typ;
    row = in.row;
    uint16_t slab = in.slab;
    const uint16_t slab0 = slab;
    const int mat = d.smat[slab];
    R T = in.T;
    double u[3] = {(double)in.u[0], (double)in.u[1], (double)in.u[2]};
    double r[3] = {in.r[0], in.r[1], in.r[2]};
    uint8_t fl = in.fl;
    R nl = in.nl;
    uint32_t step = in.step;
    const uint64_t key = in.key;
    const uint64_t event = d.row_event[row];
    const bool resumed = (fl & F_PAUSED) != 0;
    double s_phys, s_done = 0.0, h_try = 0.0;
    int n_search = 0;
    R sig;
    uint64_t w_sel = 0;
    if (resumed) {
        s_phys = d.sphys[s];
        s_done = d.sdone[s];
        h_try = d.htry[s];
        n_search = d.nsearch[s];
        sig = d.xs[s];
        pre_n = 0;
    } else {
        pre_step(d, tb, mat, typ, T, nl, event, key, step, sig, s_phys, fl, w_sel);
        pre_n = 1;
    }
    double Td = (double)T;
    double q = typ == kPositron ? 1.0 : -1.0;
    double p = sqrt(Td * (Td + 2.0 * kMe));
    double kf = q * kCk / p;
    double Bm = sqrt(d.B[0] * d.B[0] + d.B[1] * d.B[1] + d.B[2] * d.B[2]);
    double h_chord = sqrt(8.0 * kDChord / (kCk * Bm / p));
    double zlo = d.zp[slab], zhi = d.zp[slab + 1];
    int face = F_NONE;
    bool paused = false;
    for (;;) {
        if (max_sub > 0 && att >= (uint32_t)max_sub) { paused = true; break; }
        double rem = s_phys - s_done;
        double h = h_try > 0.0 ? h_try : fmin(rem, h_chord);
        bool last = (h_try == 0.0 && h == rem);
        double r1[3], u1[3];
        rk4(r, u, h, kf, d.B, r1, u1);
        ++att;
        // first face crossed by the chord r -> r1
        int fc = F_NONE;
        double f = INFINITY;
        for (int fa = F_ZLO; fa <= F_YHI; ++fa) {
            int ax = face_axis(fa);
            double pl = fa == F_ZLO ? zlo : (fa == F_ZHI ? zhi : face_plane(d.zp, slab, d.W, fa));
            if (!beyond(fa, r1[ax], pl)) continue;
            double fr = (pl - r[ax]) / (r1[ax] - r[ax]);
            fr = fr < 0.0 ? 0.0 : (fr > 1.0 ? 1.0 : fr);
            if (fr < f) { f = fr; fc = fa; }
        }
        if (fc == F_NONE) {
            int nf = F_NONE;
            if (h_try > 0.0) {
                double bd = kDInt;
                for (int fa = F_ZLO; fa <= F_YHI; ++fa) {
                    double pl = fa == F_ZLO ? zlo : (fa == F_ZHI ? zhi : face_plane(d.zp, slab, d.W, fa));
                    double dd = fabs(r1[face_axis(fa)] - pl);
                    if (dd <= bd && (nf == F_NONE || dd < bd)) { bd = dd; nf = fa; }
                }
            }
            r[0] = r1[0]; r[1] = r1[1]; r[2] = r1[2];
            normalize_d(u1);
            store_dir<R>(u1);
            u[0] = u1[0]; u[1] = u1[1]; u[2] = u1[2];
            if (nf != F_NONE) {
                r[face_axis(nf)] = face_plane(d.zp, slab, d.W, nf);
                s_done += h;
                face = nf;
                break;
            }
            if (last) { s_done = s_phys; break; }
            s_done += h;
            h_try = 0.0;
            n_search = 0;
            continue;
        }
        if (f == 0.0 && points_out(u, fc)) {
            r[face_axis(fc)] = face_plane(d.zp, slab, d.W, fc);
            face = fc;
            break;
        }
        double ch[3] = {r1[0] - r[0], r1[1] - r[1], r1[2] - r[2]};
        double clen = sqrt(ch[0] * ch[0] + ch[1] * ch[1] + ch[2] * ch[2]);
        if ((1.0 - f) * clen <= kDInt || n_search >= kMaxSearch) {
            for (int c = 0; c < 3; ++c) r[c] = r[c] + f * ch[c];
            r[face_axis(fc)] = face_plane(d.zp, slab, d.W, fc);
            normalize_d(u1);
            store_dir<R>(u1);
            u[0] = u1[0]; u[1] = u1[1]; u[2] = u1[2];
            s_done += f * h;
            face = fc;
            break;
        }
        h_try = f > 0.0 ? f * h : 0.5 * h;
        n_search += 1;
    }
    paused_n = paused ? 1u : 0u;
    if (paused) {
        // the kinetic energy changes only at the end of the step
        TrackRec<R> out;
        out.r[0] = r[0];
        out.r[1] = r[1];
        out.r[2] = r[2];
        out.key = key;
        out.u[0] = (R)u[0];
        out.u[1] = (R)u[1];
        out.u[2] = (R)u[2];
        out.T = in.T;
        store_track(d, s, out);
        d.sdone[s] = s_done;
        d.htry[s] = h_try;
        d.nsearch[s] = (uint8_t)n_search;
        d.flags[s] = fl | F_PAUSED;
        if (!resumed) {
            // the step limit, cross section and interaction length of the
            // step persist until it resumes
            d.sphys[s] = s_phys;
            d.xs[s] = sig;
            d.nl[s] = nl;
            d.action[s] = A_FIELD;
        }
        return;
    }
    fl = fl & (uint8_t)~F_PAUSED;
    StepTally tl = {0.0, 0, 0, 0};
    bool alive = true;
    uint8_t na = A_IDLE;
    const uint32_t k0 = step;
    finish_along<R, true>(d, tb, typ, T, sig, s_done, face, fl, mat, slab, tl, alive, na, nl, step, key, event, row,
                          !resumed, w_sel);
    record_tally(d, row, slab0, tl);
    if (alive) {
        if (d.msc && na != A_ANNIH) msc_deflect(d.seed, event, key, k0, Td, s_done, d.x0[mat], u);
        TrackRec<R> tr;
        tr.r[0] = r[0];
        tr.r[1] = r[1];
        tr.r[2] = r[2];
        tr.key = key;
        tr.u[0] = (R)u[0];
        tr.u[1] = (R)u[1];
        tr.u[2] = (R)u[2];
        tr.T = T;
        store_track(d, s, tr);
        d.nl[s] = nl;
        if (slab != slab0) d.slab[s] = slab;
        if (step != k0) d.step[s] = step;
        d.flags[s] = fl;
        d.action[s] = na;
        next = na;
    } else {
        retired = step;
        retire(d, s, row, retired);
    }
}

template <class R>
__device__ __forceinline__ void along_field_track(const Dev<R>& d, const Tables<R>& tb, uint32_t s, int max_sub,
                                                  uint32_t& row, uint8_t& next, uint32_t& retired, uint32_t& att,
                                                  uint32_t& paused_n, uint32_t& pre_n)
{
    FieldIn<R> in;
    load_field_in(d, s, in);
    along_field_track<R>(d, tb, s, in, max_sub, row, next, retired, att, paused_n, pre_n);
}

// Uniform-field propagation with RK4 substeps of at most sqrt(8 d_chord /
// curvature), boundary search by chord fraction, and a cap of max_substeps
// RK4 evaluations per iteration: at the cap the step pauses with its
// position, direction, path length and search state saved, and resumes in the
// next iteration (paper, "Reducing load imbalance").  Momentum is fixed during
// the step, so a paused step ends exactly as an uninterrupted one.
// Per-thread counts of the along-step kernels, flushed once per block.
struct AlongAcc {
    unsigned long long field = 0, photon = 0, ret_field = 0, ret_photon = 0, sub = 0, pause = 0, pre = 0;
};

// One field track's along-step from its loaded inputs, with the counts.
template <class R>
__device__ __forceinline__ void field_step_loaded(const Dev<R>& d, const Tables<R>& tb, uint32_t s,
                                                  const FieldIn<R>& in, bool act, AlongAcc& acc)
{
    uint32_t row = 0;
    uint8_t next = A_NONE;
    uint32_t retired = 0, att = 0, paused_n = 0, pre_n = 0;
    if (act) along_field_track<R>(d, tb, s, in, d.max_substeps, row, next, retired, att, paused_n, pre_n);
    acc.field += act ? 1u : 0u;
    acc.pre += pre_n;
    leave_event(d, retired != 0, row);
    acc.ret_field += retired;
    acc.sub += att;
    acc.pause += paused_n;
    if (d.sorted2 == 2 && (d.ctr->phase_sorted & 2u)) append_to_list(d, next >= A_PROC0 && next < A_NUM, next, s);
}

// The field tracks of a sorted iteration, positions [0, n) of the
// permutation from `off`: each thread walks its positions at the grid
// stride and loads the next track's fields (and the slot after it) before
// stepping the current one, so those loads are in flight during the step.
template <class R>
__device__ __forceinline__ void field_tracks_sorted(const Dev<R>& d, const Tables<R>& tb, uint32_t n, uint32_t off,
                                                    AlongAcc& acc)
{
    const uint32_t stride = gridDim.x * blockDim.x;
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t s = i < n ? d.perm[off + i] : 0u;
    FieldIn<R> cur;
    if (i < n) load_field_in(d, s, cur);
    uint32_t s_next = i + stride < n ? d.perm[off + i + stride] : 0u;
    for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += stride) {
        const bool act = i < n;
        const uint32_t i1 = i + stride, i2 = i + 2 * stride;
        FieldIn<R> nxt;
        if (i1 < n) load_field_in(d, s_next, nxt);
        const uint32_t s_after = i2 < n ? d.perm[off + i2] : 0u;
        field_step_loaded(d, tb, s, cur, act, acc);
        i = i1;
        s = s_next;
        cur = nxt;
        s_next = s_after;
    }
}

// One track's along-step by its along action (masked iterations).
template <class R>
__device__ __forceinline__ void along_any_track(const Dev<R>& d, const Tables<R>& tb, uint32_t s, uint8_t a,
                                                AlongAcc& acc)
{
    uint32_t row = 0;
    uint8_t next = A_NONE;
    uint32_t retired = 0, att = 0, paused_n = 0, pre_n = 0;
    if (a == A_FIELD) {
        along_field_track<R>(d, tb, s, d.max_substeps, row, next, retired, att, paused_n, pre_n);
        ++acc.field;
        acc.ret_field += retired;
    } else if (a == A_NEUTRAL) {
        along_straight_track<R, false>(d, tb, s, row, next, retired);
        pre_n = 1;
        ++acc.photon;
        acc.ret_photon += retired;
    }
    acc.pre += pre_n;
    acc.sub += att;
    acc.pause += paused_n;
    leave_event(d, retired != 0, row);
    if (d.sorted2 == 2 && (d.ctr->phase_sorted & 2u)) append_to_list(d, next >= A_PROC0 && next < A_NUM, next, s);
}

template <class R>
__global__ void __launch_bounds__(kStepMaxBlock) k_along_field(Dev<R> d)
{
    extern __shared__ __align__(16) unsigned char ems_lds[];
    EMS_TRACK_RANGE(d, A_FIELD)
    const Tables<R> tb = block_tables(d, (R*)ems_lds);
    AlongAcc acc;
    if (_mode == 1) {
        field_tracks_sorted(d, tb, _n, _off, acc);
    } else {
        EMS_FOR_TRACKS(d, A_FIELD, s, act, W_FIELD)
        along_any_track(d, tb, s, act ? (uint8_t)A_FIELD : (uint8_t)A_NONE, acc);
        EMS_END_TRACKS
        (void)_work;                 // the same count as acc.field
    }
    flush_count(d, W_FIELD, acc.field);
    flush_count(d, kStepsSlot + W_FIELD, acc.ret_field);
    flush_count(d, W_SUBSTEPS, acc.sub);
    flush_count(d, W_PAUSED, acc.pause);
    flush_count_shared(d, W_PRE, acc.pre);
}

// Both along-steps of a field iteration in one launch (tuning `fuse_along`):
// sorted, each thread first steps its field tracks as k_along_field does,
// then its share of the photon range, which is dealt out starting at the
// waves that had one field round fewer, so that the photon steps fill the
// end of the field launch instead of paying for a launch of their own.
// Masked, each slot takes the along-step of its type.
template <class R>
__global__ void __launch_bounds__(kStepMaxBlock) k_along_both(Dev<R> d)
{
    extern __shared__ __align__(16) unsigned char ems_lds[];
    const int mode = (d.ctr->phase_sorted & 1u) ? d.sorted : 0;
    const uint32_t nf = mode == 1 ? d.ctr->range_cnt[A_FIELD] : d.n_slots;
    const uint32_t np = mode == 1 ? d.ctr->range_cnt[A_NEUTRAL] : 0u;
    // sorted, every wave of the grid may be dealt photon chunks: no early exit
    // (masked, the grid never exceeds the slots)
    if (mode != 1 && blockIdx.x * blockDim.x >= nf) return;          // block-uniform
    const Tables<R> tb = block_tables(d, (R*)ems_lds);
    AlongAcc acc;
    if (mode == 1) {
        field_tracks_sorted(d, tb, nf, d.ctr->range_off[A_FIELD], acc);
        // photon chunks of 64 positions: chunk c goes to wave (r + c) mod W,
        // r = the number of waves that took one field round more
        const uint32_t waves = gridDim.x * blockDim.x / 64;
        const uint32_t w = (blockIdx.x * blockDim.x + threadIdx.x) / 64;
        const uint32_t r = (nf / 64 + (nf % 64 != 0)) % waves;
        const uint32_t first = (w + waves - r) % waves;
        const uint32_t offp = d.ctr->range_off[A_NEUTRAL];
        for (uint32_t c = first; (size_t)c * 64 < np; c += waves) {
            const uint32_t j = c * 64 + lane_id();
            const bool act = j < np;
            along_any_track(d, tb, act ? d.perm[offp + j] : 0u, act ? (uint8_t)A_NEUTRAL : (uint8_t)A_NONE, acc);
        }
    } else {
        // masked: each thread walks its positions at the grid stride -- the
        // slots, or with compact_along the slots occupied before the fill
        // (in slot order) followed by the vacancies the fill used (the
        // lowest n_take_lo, then the highest) -- and steps each slot's own
        // type; the along action of the position after next and the inputs
        // of the next one, if it holds a field track, are loaded before the
        // current one steps
        const Counters* c = d.ctr;
        const uint32_t n_old = c->alive_before, n_take = c->n_take_q + c->n_take_p;
        // the listed walk pays when most slots are empty; when most are
        // occupied the plain walk reads each line once, where the listed one
        // reaches a line from both lists
        const bool cl = d.compact_along != 0 && 2 * (n_old + n_take) < nf;
        const uint32_t n_lo = c->n_take_lo, n_vac = c->n_vac;
        const uint32_t np_all = cl ? n_old + n_take : nf;
        auto slot_at = [&](uint32_t p) -> uint32_t {
            if (!cl) return p;
            if (p < n_old) return d.along_list[p];
            const uint32_t q = p - n_old;
            return q < n_lo ? d.vac[q] : d.vac[n_vac - n_take + q];
        };
        const uint32_t stride = gridDim.x * blockDim.x;
        uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
        uint32_t s = p < np_all ? slot_at(p) : 0u;
        uint32_t s1 = p + stride < np_all ? slot_at(p + stride) : 0u;
        uint8_t a = p < np_all ? along_action(d, s) : A_NONE;
        uint8_t a1 = p + stride < np_all ? along_action(d, s1) : A_NONE;
        FieldIn<R> cur;
        if (a == A_FIELD) load_field_in(d, s, cur);
        for (uint32_t base = blockIdx.x * blockDim.x; base < np_all; base += stride) {
            const uint32_t p2 = p + 2 * stride;
            FieldIn<R> nxt;
            if (a1 == A_FIELD) load_field_in(d, s1, nxt);
            const uint32_t s2 = p2 < np_all ? slot_at(p2) : 0u;
            const uint8_t a2 = p2 < np_all ? along_action(d, s2) : A_NONE;
            if (a == A_FIELD) field_step_loaded(d, tb, s, cur, true, acc);
            else along_any_track(d, tb, s, a, acc);
            p += stride;
            s = s1;
            s1 = s2;
            a = a1;
            a1 = a2;
            cur = nxt;
        }
    }
    flush_count(d, W_FIELD, acc.field);
    flush_count(d, W_NEUTRAL, acc.photon);
    flush_count(d, kStepsSlot + W_FIELD, acc.ret_field);
    flush_count(d, kStepsSlot + W_NEUTRAL, acc.ret_photon);
    flush_count(d, W_SUBSTEPS, acc.sub);
    flush_count(d, W_PAUSED, acc.pause);
    flush_count_shared(d, W_PRE, acc.pre);
}

// Discrete interaction PROC of one track at the end of its along-step.
// Outputs as for the along-step (the secondaries start at the track's point).
template <class R, int PROC>
__device__ __forceinline__ void interact_track(const Dev<R>& d, uint32_t s, SecBuf<R>& sb, double r[3], uint32_t& row,
                                               uint16_t& slab, uint32_t& retired)
{
    row = d.row[s];
    slab = d.slab[s];
    const TrackRec<R> tr = load_track(d, s);
    r[0] = tr.r[0]; r[1] = tr.r[1]; r[2] = tr.r[2];
    Prim<R> p;
    p.T = tr.T;
    p.u[0] = tr.u[0]; p.u[1] = tr.u[1]; p.u[2] = tr.u[2];
    p.key = tr.key;
    p.step = d.step[s];
    p.type = d.type[s];
    p.alive = true;
    uint8_t fl = d.flags[s];
    PhysParams pp = {d.seed, d.row_event[row], d.ecut};
    StepRng<R> rng(d.seed, pp.event, p.key, p.step, (fl & F_DREW) ? 2 : 1);
    StepTally tl = {0.0, 0, 0, 0};
    switch (PROC) {
    case P_COMPTON: sample_compton<R>(pp, p, rng, sb, tl); break;
    case P_PHOTO:   sample_photo<R>(pp, p, sb, tl); break;
    case P_PAIR:    sample_pair<R>(pp, p, rng, sb, tl); break;
    case P_MOLLER:  sample_moller<R>(pp, p, rng, sb, tl); break;
    case P_BHABHA:  sample_bhabha<R>(pp, p, rng, sb, tl); break;
    case P_BREMS:   sample_brems<R>(pp, p, rng, sb, tl); break;
    default:
        // at rest (the kinetic energy was deposited by the along-step)
        annihilate<R>(pp, p.key, p.step, sb, tl);
        p.T = R(0);
        p.alive = false;
        break;
    }
    // a step-guard stop was counted by the along-step already
    uint32_t steps = (PROC == P_ANNIH && (fl & F_COUNTED)) ? p.step : p.step + 1;
    d.step[s] = steps;
    if (p.alive && steps > kMaxSteps) {
        atomicAdd(&ledger_of(d, row).n_guard, 1ull);
        p.step = steps;
        if (p.type != kGamma) stop_lepton<R>(pp, p, sb, tl);
        else { tl.edep += (double)p.T; p.alive = false; }
    }
    record_tally(d, row, slab, tl);
    if (p.alive) {
        TrackRec<R> out;
        out.r[0] = r[0];
        out.r[1] = r[1];
        out.r[2] = r[2];
        out.key = p.key;
        out.u[0] = p.u[0];
        out.u[1] = p.u[1];
        out.u[2] = p.u[2];
        out.T = p.T;
        store_track(d, s, out);
        d.nl[s] = R(-1);
        d.action[s] = A_IDLE;
    } else {
        retired = steps;
        retire(d, s, row, steps);
    }
}

// ---- discrete interactions: one kernel per process ---------------------------------
template <class R, int PROC, bool DET>
__global__ void __launch_bounds__(kStepMaxBlock) k_interact(Dev<R> d)
{
    EMS_TRACK_RANGE(d, (uint8_t)(A_PROC0 + PROC))
    unsigned long long ret_acc = 0, reuse_acc = 0;
    EMS_FOR_TRACKS(d, (uint8_t)(A_PROC0 + PROC), s, act, W_PROC0 + PROC)
    SecBuf<R> sb;
    sb.n = 0;
    double r[3] = {0.0, 0.0, 0.0};
    uint32_t row = 0;
    uint16_t slab = 0;
    uint32_t retired = 0;
    if (act) interact_track<R, PROC>(d, s, sb, r, row, slab, retired);
    if (retired) reuse_acc += reuse_slot(d, s, sb, row, slab, r);
    append_secondaries<R, DET>(d, sb, row, slab, r, retired != 0, _off + _i);
    ret_acc += retired;
    EMS_END_TRACKS
    flush_count(d, W_PROC0 + PROC, _work);
    flush_count(d, kStepsSlot + W_PROC0 + PROC, ret_acc);
    flush_count_shared(d, W_REUSE, reuse_acc);
}

// ---- discrete interactions, all seven actions in one launch ------------------------
// After the reordering at sort point 2 the seven interaction actions (six
// processes and annihilation at rest) occupy consecutive index ranges of the
// permutation (or seven lists), so one launch
// can walk all of them: each wave then holds one process except at the few
// range boundaries.  The per-track code is that of the per-process kernels;
// the launch count per iteration drops from seven to one.  Unsorted, it masks
// over all slots like the per-process kernels.
template <class R, bool DET>
__global__ void __launch_bounds__(kStepMaxBlock) k_interact_all(Dev<R> d)
{
    const int mode = (d.ctr->phase_sorted & 2u) ? d.sorted2 : 0;
    uint32_t n = d.n_slots, off = 0;
    uint32_t lc0 = 0, lc1 = 0, lc2 = 0, lc3 = 0, lc4 = 0, lc5 = 0;
    if (mode == 1) {
        off = d.ctr->range_off[A_PROC0];
        n = d.ctr->range_off[A_ANNIH] + d.ctr->range_cnt[A_ANNIH] - off;
        // ends of the first six action ranges, relative to the first
        lc0 = d.ctr->range_off[A_PROC0 + 1] - off;
        lc1 = d.ctr->range_off[A_PROC0 + 2] - off;
        lc2 = d.ctr->range_off[A_PROC0 + 3] - off;
        lc3 = d.ctr->range_off[A_PROC0 + 4] - off;
        lc4 = d.ctr->range_off[A_PROC0 + 5] - off;
        lc5 = d.ctr->range_off[A_PROC0 + 6] - off;
    } else if (mode == 2) {
        lc0 = d.ctr->list_cnt[A_PROC0];
        lc1 = lc0 + d.ctr->list_cnt[A_PROC0 + 1];
        lc2 = lc1 + d.ctr->list_cnt[A_PROC0 + 2];
        lc3 = lc2 + d.ctr->list_cnt[A_PROC0 + 3];
        lc4 = lc3 + d.ctr->list_cnt[A_PROC0 + 4];
        lc5 = lc4 + d.ctr->list_cnt[A_PROC0 + 5];
        n = lc5 + d.ctr->list_cnt[A_PROC0 + 6];
    }
    if (blockIdx.x * blockDim.x >= n) return;
    unsigned long long w0 = 0, w1 = 0, w2 = 0, w3 = 0, w4 = 0, w5 = 0, w6 = 0, ret_acc = 0, reuse_acc = 0;
    for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
        const uint32_t i = base + threadIdx.x;
        bool act = i < n;
        uint32_t s = 0;
        uint8_t a = A_NONE;
        if (act) {
            // sorted: the process follows from the position in the ranges
            const int p = i < lc0 ? 0 : (i < lc1 ? 1 : (i < lc2 ? 2 : (i < lc3 ? 3 : (i < lc4 ? 4 : (i < lc5 ? 5 : 6)))));
            if (mode == 1) {
                s = d.perm[off + i];
                a = (uint8_t)(A_PROC0 + p);
            } else if (mode == 2) {
                uint32_t lo = p == 0 ? 0u
                                     : (p == 1 ? lc0 : (p == 2 ? lc1 : (p == 3 ? lc2 : (p == 4 ? lc3 : (p == 5 ? lc4 : lc5)))));
                s = d.lists[(size_t)(A_PROC0 + p) * d.n_slots + (i - lo)];
                a = (uint8_t)(A_PROC0 + p);
            } else {
                s = i;
                a = d.action[s];
            }
        }
        act = act && a >= A_PROC0 && a < A_NUM;
        SecBuf<R> sb;
        sb.n = 0;
        double r[3] = {0.0, 0.0, 0.0};
        uint32_t row = 0;
        uint16_t slab = 0;
        uint32_t retired = 0;
        if (act) {
            switch (a - A_PROC0) {
            case P_COMPTON: interact_track<R, P_COMPTON>(d, s, sb, r, row, slab, retired); ++w0; break;
            case P_PHOTO:   interact_track<R, P_PHOTO>(d, s, sb, r, row, slab, retired); ++w1; break;
            case P_PAIR:    interact_track<R, P_PAIR>(d, s, sb, r, row, slab, retired); ++w2; break;
            case P_MOLLER:  interact_track<R, P_MOLLER>(d, s, sb, r, row, slab, retired); ++w3; break;
            case P_BHABHA:  interact_track<R, P_BHABHA>(d, s, sb, r, row, slab, retired); ++w4; break;
            case P_BREMS:   interact_track<R, P_BREMS>(d, s, sb, r, row, slab, retired); ++w5; break;
            default:        interact_track<R, P_ANNIH>(d, s, sb, r, row, slab, retired); ++w6; break;
            }
        }
        if (retired) reuse_acc += reuse_slot(d, s, sb, row, slab, r);
        append_secondaries<R, DET>(d, sb, row, slab, r, retired != 0, off + i);
        ret_acc += retired;
    }
    flush_count(d, W_PROC0 + P_COMPTON, w0);
    flush_count(d, W_PROC0 + P_PHOTO, w1);
    flush_count(d, W_PROC0 + P_PAIR, w2);
    flush_count(d, W_PROC0 + P_MOLLER, w3);
    flush_count(d, W_PROC0 + P_BHABHA, w4);
    flush_count(d, W_PROC0 + P_BREMS, w5);
    flush_count(d, W_PROC0 + P_ANNIH, w6);
    flush_count(d, kStepsSlot + W_PROC0, ret_acc);
    flush_count_shared(d, W_REUSE, reuse_acc);
}

// ---- drain: block-local stepping of the last tracks ---------------------------------
// When few tracks are left the step loop is bound by per-iteration launch
// latency, not by work.  A drain launch steps them without further launches:
// each block runs its own small step loop in rounds.  Half of a block's
// threads own occupied slots, half own vacant ones; in every round each
// thread with a track takes up to kDrainBurst steps -- pre-step, along-step
// and interaction, through the same per-track functions as the action
// kernels -- and the secondaries go onto the block's stack (LIFO); at the
// start of the next round the threads whose slot is vacant take the newest
// entries.  A sub-shower so spreads over the block's threads instead of one
// thread stepping it alone.  A thread knows from its own steps whether its
// slot holds a track (a step that retires the track says so), so a round
// reads no slot state beyond what the steps read; several steps per round
// spread the round's barriers over them, which matters at the end, when a
// few long-lived tracks are left.
// After `max_steps` rounds, or when a block has neither tracks nor entries,
// the block stops; its stack entries (and any that did not fit) go to the
// initializer buffer for the step loop.  Random numbers are keyed by track
// and step, so every track ends exactly as in the step loop.

// Secondaries of one step onto the block's stack while it has room (`top`
// counts its entries, in LDS), else to the initializer buffer.
template <class R>
__device__ __forceinline__ void drain_push(const Dev<R>& d, const SecBuf<R>& sb, uint32_t row, uint16_t slab,
                                           const double r[3], Initializer* bstack, int cap, int* top, bool retiring)
{
    // the event's counters change once per track, as in append_secondaries
    const int dlive = sb.n - (retiring ? 1 : 0);
    if (dlive != 0) atomicAdd(live_of(d, row), (unsigned int)dlive);    // modulo 2^32: a decrement for -1
    if (sb.n == 0) return;
    const int pos = atomicAdd(top, sb.n);
    unsigned int n_gam = 0, n_ele = 0, n_pos = 0;
    sb.each([&](const Sec<R>& v, int k) {
        Initializer rec;
        rec.T = (double)v.T;
        rec.r[0] = r[0]; rec.r[1] = r[1]; rec.r[2] = r[2];
        rec.u[0] = (double)v.ux; rec.u[1] = (double)v.uy; rec.u[2] = (double)v.uz;
        rec.key = v.key;
        rec.row = row;
        rec.slab = slab;
        rec.type = (uint8_t)v.type;
        rec.pad = 0;
        n_gam += v.type == kGamma;
        n_ele += v.type == kElectron;
        n_pos += v.type == kPositron;
        if (pos + k < cap) {
            bstack[pos + k] = rec;
        } else {
            unsigned long long q = atomicAdd(&d.ctr->queue_size, 1ull);
            if (q < d.queue_cap) d.queue[q] = rec;
            else atomicOr(&d.ctr->overflow, 1u);
        }
    });
    if (n_gam) atomicAdd(&ledger_of(d, row).n_sec[kGamma], (unsigned long long)n_gam);
    if (n_ele) atomicAdd(&ledger_of(d, row).n_sec[kElectron], (unsigned long long)n_ele);
    if (n_pos) atomicAdd(&ledger_of(d, row).n_sec[kPositron], (unsigned long long)n_pos);
}

// Exclusive rank of a true flag among the block's threads, and their total.
// Contains a barrier (all threads of the block must call it).
__device__ __forceinline__ uint32_t block_rank(bool f, uint32_t* wcnt, uint32_t& total)
{
    const uint64_t m = __ballot(f);
    const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    if (lane_id() == 0) wcnt[w] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t r = rank_below(m), tot = 0;
    for (int i = 0; i < nw; ++i) {
        if (i < w) r += wcnt[i];
        tot += wcnt[i];
    }
    total = tot;
    return r;
}

template <class R>
__device__ __forceinline__ void drain_interact(const Dev<R>& d, int proc, uint32_t s, SecBuf<R>& sb, double r[3],
                                               uint32_t& row, uint16_t& slab, uint32_t& retired)
{
    switch (proc) {
    case P_COMPTON: interact_track<R, P_COMPTON>(d, s, sb, r, row, slab, retired); break;
    case P_PHOTO:   interact_track<R, P_PHOTO>(d, s, sb, r, row, slab, retired); break;
    case P_PAIR:    interact_track<R, P_PAIR>(d, s, sb, r, row, slab, retired); break;
    case P_MOLLER:  interact_track<R, P_MOLLER>(d, s, sb, r, row, slab, retired); break;
    case P_BHABHA:  interact_track<R, P_BHABHA>(d, s, sb, r, row, slab, retired); break;
    case P_BREMS:   interact_track<R, P_BREMS>(d, s, sb, r, row, slab, retired); break;
    default:        interact_track<R, P_ANNIH>(d, s, sb, r, row, slab, retired); break;
    }
}

// Slots: O = the occupied ones (listed by the vacancy pass, then the
// vacancies just filled), E = the vacancies left empty.  In block b, thread i
// < 128 owns O[128 b + i] and thread 128 + i owns E[128 b + i] (when they
// exist), so every block has tracks and room for their secondaries.
template <class R>
__global__ void __launch_bounds__(256) k_drain(Dev<R> d, const uint32_t* live_list, Initializer* stack,
                                               uint32_t n_threads, int depth, uint32_t max_steps)
{
    extern __shared__ __align__(16) unsigned char ems_lds[];
    __shared__ int top;
    __shared__ uint32_t wcnt[4];
    const Tables<R> tb = block_tables(d, (R*)ems_lds);
    const uint32_t n_old = d.ctr->alive_before;
    const uint32_t n_take = d.ctr->n_take_q + d.ctr->n_take_p;
    const uint32_t n_occ = n_old + n_take;
    const uint32_t n_empty = d.ctr->n_vac - n_take;
    const int cap = depth * (int)blockDim.x;
    Initializer* bstack = stack + (size_t)blockIdx.x * cap;
    const uint32_t half = blockDim.x / 2;
    const uint32_t j = blockIdx.x * half + (threadIdx.x % half);
    bool owns = blockIdx.x * blockDim.x + threadIdx.x < n_threads;
    uint32_t s = 0;
    if (threadIdx.x < half) {
        owns = owns && j < n_occ;
        if (owns) s = j < n_old ? live_list[j] : d.vac[j - n_old];
    } else {
        owns = owns && j < n_empty;
        if (owns) s = d.vac[n_take + j];
    }
    unsigned long long ret_acc = 0, work = 0;
    bool has = owns && d.type[s] != kDead;     // the thread's slot holds a track
    if (threadIdx.x == 0) top = 0;
    __syncthreads();
    for (uint32_t k = 0; k < max_steps; ++k) {
        // threads with a vacant slot take the newest entries of the stack
        const bool idle = owns && !has;
        uint32_t n_idle = 0;
        const uint32_t rank = block_rank(idle, wcnt, n_idle);
        const int avail = top;
        if (idle && (int)rank < avail) {
            init_slot(d, s, bstack[avail - 1 - (int)rank]);
            has = true;
        }
        __syncthreads();
        if (threadIdx.x == 0) top = avail - ((int)n_idle < avail ? (int)n_idle : avail);
        // no track left in the block: then its stack is empty too
        if (!__syncthreads_or(has)) break;
        for (int burst = 0; burst < kDrainBurst && has; ++burst) {
            // the along-step functions run the pre-step (a paused step is a
            // field step and resumes without one)
            const uint8_t a = along_action(d, s);
            if (a == A_NONE) {      // (every retirement is reported; kept as a guard)
                has = false;
                break;
            }
            uint32_t row = 0, retired = 0;
            uint8_t next = A_NONE;
            if (a == A_NEUTRAL) {
                along_straight_track<R, false>(d, tb, s, row, next, retired);
            } else if (a == A_CHARGED) {
                along_straight_track<R, true>(d, tb, s, row, next, retired);
            } else {
                // a paused step resumes at the thread's next step (pausing does not change the result)
                uint32_t att = 0, paused_n = 0, pre_n = 0;
                along_field_track<R>(d, tb, s, kDrainSubsteps, row, next, retired, att, paused_n, pre_n);
            }
            if (next >= A_PROC0 && next < A_NUM) {
                SecBuf<R> sb;
                sb.n = 0;
                double r[3] = {0.0, 0.0, 0.0};
                uint16_t slab = 0;
                drain_interact<R>(d, next - A_PROC0, s, sb, r, row, slab, retired);
                drain_push(d, sb, row, slab, r, bstack, cap, &top, retired != 0);
            } else if (retired) {
                leave_event(d, true, row);
            }
            ret_acc += retired;
            ++work;
            has = retired == 0;     // a retired track has left its slot
        }
        __syncthreads();
        if (threadIdx.x == 0 && top > cap) top = cap;     // the excess went to the initializer buffer
        __syncthreads();
    }
    // what is left on the stack goes back to the step loop
    const int left = top;
    for (int i = threadIdx.x; i < left; i += blockDim.x) {
        unsigned long long q = atomicAdd(&d.ctr->queue_size, 1ull);
        if (q < d.queue_cap) d.queue[q] = bstack[i];
        else atomicOr(&d.ctr->overflow, 1u);
    }
    flush_count(d, W_DRAIN, work);
    flush_count(d, kStepsSlot + W_DRAIN, ret_acc);
}

// ---- event completion ---------------------------------------------------------------
// After an iteration, an occupied row whose live count is zero has finished:
// record it once in the completion ring (entries carry the row's generation).
template <class R>
__global__ void k_scan_completions(Dev<R> d)
{
    uint32_t row = blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= d.n_rows) return;
    unsigned int live = 0;          // modulo 2^32: a copy can hold a net decrement
    for (uint32_t r = 0; r <= d.rep_mask; ++r) live += d.live[(size_t)r * d.live_rs + row];
    if (d.row_state[row] == 1u && live == 0u) {
        d.row_state[row] = 0u;
        unsigned int k = atomicAdd(&d.ctr->done_count, 1u);
        d.done_ring[k % d.n_rows] = ((unsigned long long)d.row_gen[row] << 32) | row;
    }
}

// ---- stable counting sort of slot indices by a small key ----------------------------
// Sort key of a slot at a sort point; 0xFF excludes the slot.
//   keymode 0 (partition): the next action (< 16)
//   keymode 1 (radix): action << 3 | type << 1 | (material & 1) (< 128)
//   keymodes 2 and 3: as 0 and 1 with the along-step action from the type
//   (the first sort, before the along-step kernels run the pre-step)
template <class R>
__device__ __forceinline__ uint32_t sort_key(const Dev<R>& d, uint32_t s, int keymode)
{
    uint8_t a = keymode >= 2 ? along_action(d, s) : d.action[s];
    if (a == A_NONE || a == A_IDLE) return 0xFFu;
    if (keymode == 0 || keymode == 2) return a;
    uint32_t t = d.type[s];
    uint32_t m = (uint32_t)d.smat[d.slab[s]] & 1u;
    return ((uint32_t)a << 3) | (t << 1) | m;
}


// Per-tile histogram: cnt[bin * n_tiles + tile]
template <class R, int NB>
__global__ void __launch_bounds__(kSortThreads) k_sort_hist(Dev<R> d, int keymode, const uint8_t* ext_keys, uint32_t n,
                                                            uint32_t* cnt, uint32_t n_tiles)
{
    if (!ext_keys && !(d.ctr->phase_sorted & (keymode >= 2 ? 1u : 2u))) return;
    __shared__ uint32_t h[NB];
    for (int b = threadIdx.x; b < NB; b += kSortThreads) h[b] = 0;
    __syncthreads();
    uint32_t base = blockIdx.x * kSortTile;
    for (int k = threadIdx.x; k < kSortTile; k += kSortThreads) {
        uint32_t i = base + k;
        if (i >= n) break;
        uint32_t key = ext_keys ? ext_keys[i] : sort_key(d, i, keymode);
        if (key < NB) atomicAdd(&h[key], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < NB; b += kSortThreads) cnt[b * n_tiles + blockIdx.x] = h[b];
}

// Per-bin exclusive scan of the tile counts: block `bin` scans cnt[bin][*]
// in place (tile order) and writes the bin's total.
template <int NB>
__global__ void __launch_bounds__(256) k_sort_scan(uint32_t* cnt, uint32_t n_tiles, const Counters* ctr,
                                                   uint32_t* bin_total, unsigned int phase_bit)
{
    if (ctr && !(ctr->phase_sorted & phase_bit)) return;
    __shared__ uint32_t wsum[4];
    const uint32_t bin = blockIdx.x;
    uint32_t* c = cnt + (size_t)bin * n_tiles;
    const uint32_t per = (n_tiles + 255) / 256;
    const uint32_t t0 = threadIdx.x * per, t1 = t0 + per < n_tiles ? t0 + per : n_tiles;
    uint32_t local = 0;
    for (uint32_t t = t0; t < t1; ++t) local += c[t];
    // block-wide exclusive scan of the per-thread sums
    const int lane = lane_id(), w = threadIdx.x >> 6;
    uint32_t x = local;
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    uint32_t before = 0;
    for (int i = 0; i < w; ++i) before += wsum[i];
    uint32_t run = before + x - local;
    for (uint32_t t = t0; t < t1; ++t) {
        uint32_t v = c[t];
        c[t] = run;
        run += v;
    }
    if (threadIdx.x == 255) bin_total[bin] = before + x;
}

// Stable scatter: within a tile, items keep index order per key (wave
// ballots rank lanes of equal key; waves and rounds are ordered through LDS).
template <class R, int NB>
__global__ void __launch_bounds__(kSortThreads) k_sort_scatter(Dev<R> d, int keymode, const uint8_t* ext_keys,
                                                               uint32_t n, const uint32_t* cnt, uint32_t n_tiles,
                                                               const uint32_t* bin_total, uint32_t* perm)
{
    if (!ext_keys && !(d.ctr->phase_sorted & (keymode >= 2 ? 1u : 2u))) return;
    constexpr int NW = kSortThreads / 64;
    __shared__ uint32_t run[NB];
    __shared__ uint32_t bbase[NB + 1];
    __shared__ uint32_t wc[NW][NB];
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int b = 0; b < NB; ++b) {
            bbase[b] = acc;
            acc += bin_total[b];
        }
        bbase[NB] = acc;
    }
    __syncthreads();
    for (int b = threadIdx.x; b < NB; b += kSortThreads) run[b] = bbase[b] + cnt[b * n_tiles + blockIdx.x];
    if (!ext_keys && blockIdx.x == 0 && threadIdx.x < 16) {
        // index range of each action in the sorted permutation
        uint32_t a = threadIdx.x;
        const bool by_action = keymode == 0 || keymode == 2;
        uint32_t lo_bin = by_action ? a : a << 3;
        uint32_t hi_bin = by_action ? a + 1 : (a + 1) << 3;
        if (lo_bin >= (uint32_t)NB) {
            d.ctr->range_off[a] = bbase[NB];
            d.ctr->range_cnt[a] = 0;
        } else {
            uint32_t end = hi_bin < (uint32_t)NB ? bbase[hi_bin] : bbase[NB];
            d.ctr->range_off[a] = bbase[lo_bin];
            d.ctr->range_cnt[a] = end - bbase[lo_bin];
        }
    }
    for (int b = threadIdx.x; b < NW * NB; b += kSortThreads) (&wc[0][0])[b] = 0;
    __syncthreads();
    int w = threadIdx.x >> 6;
    int lane = lane_id();
    uint32_t base = blockIdx.x * kSortTile;
    for (int round = 0; round < kSortTile / kSortThreads; ++round) {
        uint32_t i = base + round * kSortThreads + threadIdx.x;
        uint32_t key = 0xFFFFFFFFu;
        if (i < n) key = ext_keys ? ext_keys[i] : sort_key(d, i, keymode);
        bool valid = key < (uint32_t)NB;
        // rank among equal keys in this wave
        uint32_t my_rank = 0;
        uint64_t pending = __ballot(valid);
        while (pending) {
            int leader = __ffsll((long long)pending) - 1;
            uint32_t lk = __shfl(key, leader, 64);
            uint64_t same = __ballot(valid && key == lk);
            if (valid && key == lk) my_rank = rank_below(same);
            if (lane == leader) wc[w][lk] = (uint32_t)__popcll(same);
            pending &= ~same;
        }
        __syncthreads();
        if (valid) {
            uint32_t pos = run[key] + my_rank;
            for (int k = 0; k < w; ++k) pos += wc[k][key];
            if (pos < n) perm[pos] = i;     // always in range when the tile counts match the keys
        }
        __syncthreads();
        for (int b = threadIdx.x; b < NB; b += kSortThreads) {
            uint32_t add = 0;
            for (int k = 0; k < NW; ++k) { add += wc[k][b]; wc[k][b] = 0; }
            run[b] += add;
        }
        __syncthreads();
    }
}

}  // namespace ems
