// Host driver and C ABI of the step-based EM shower transport library.
//
// The host runs the outer loop of step iterations (paper, "Stepping
// algorithm"); each iteration launches, in stream order:
//   vacancy count / scatter  -> initialization (optionally partitioned)
//   -> [sort point 1, by the along-step action of each type]
//   -> pre-step and along-step (neutral, charged, field; one kernel each)
//   -> [sort point 2] -> seven interaction kernels, or one fused launch;
// after each launch group, a completion scan.
// Below a live-track threshold ems_run replaces the iteration by a fill and
// one drain launch (block-local step loops).  Loop termination is read from device
// counters copied asynchronously to a pinned host buffer after every batch of
// iterations; batches can be captured once into a HIP graph and replayed.  No
// synchronous memory operation is issued inside the loop (paper,
// "Asynchronous memory management").
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/emstep.h"
#include "common.hpp"
#include "kernels.hpp"
#include "tables_build.hpp"

using namespace ems;

namespace {

thread_local std::string g_err;

ems_status fail(ems_status s, const std::string& msg)
{
    g_err = msg;
    return s;
}

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t _e = (expr);                                                                \
        if (_e != hipSuccess)                                                                  \
            return fail(EMS_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e));   \
    } while (0)

inline uint64_t align_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

constexpr uint64_t kStagingCap = 1 << 16;   // primaries / row registrations per host-to-device copy
constexpr uint32_t kMaxCounterCopies = 64;   // copies of the per-event counters (a power of two)

// a new event row: {event id, row, registration generation}
struct RowReg {
    uint64_t ev;
    uint32_t row, gen;
};

// Workspace layout: every region 256-byte aligned, offsets from the base.
struct Layout {
    uint64_t type, action, flags, nsearch, slab, row, step, trk, nl, xs, sphys, sdone, htry;
    uint64_t queue, prims, vac, vac_cnt, init_cnt, perm, lists, sort_cnt, bin_off, ctr;
    uint64_t tables64, tables32, mats, zp, smat, row_event, edep, ledger, live, done_ring, row_gen, row_state, part, incr;
    uint64_t drain_stack, regs, x0, rowsum, ledger_out;
    uint32_t n_rep, ledger_rs, live_rs;   // copies of the per-event counters, rows per copy
    uint32_t n_rep_e;                      // copies of the deposit tallies
    uint64_t edep_rs, edep_out;            // doubles per copy; summed tallies for readers
    uint64_t sec_cnt, sec_blk, sec_rec;    // deterministic appends (staging; 0 when off)
    uint64_t along_list;                   // occupied slots before the fill (masked one-launch along-steps)
    uint32_t part_stride;
    uint32_t drain_threads;   // capacity of the drain kernel (threads; 8 stack records each)
    uint64_t total;
    uint32_t n_tiles;
};

Layout make_layout(const ems_options& o)
{
    Layout L{};
    uint64_t off = 0;
    const uint64_t n = o.n_slots;
    const uint64_t rb = o.precision == EMS_MIXED ? 4 : 8;
    auto take = [&](uint64_t bytes) {
        uint64_t at = off;
        off = align_up(off + bytes, 256);
        return at;
    };
    L.type = take(n);
    L.action = take(n);
    L.flags = take(n);
    L.nsearch = take(n);
    L.slab = take(2 * n);
    L.row = take(4 * n);
    L.step = take(4 * n);
    L.trk = take(kTrackRec * n);
    L.nl = take(rb * n);
    L.xs = take(rb * n);
    L.sphys = take(8 * n);
    L.sdone = take(8 * n);
    L.htry = take(8 * n);
    L.queue = take(sizeof(Initializer) * o.n_initializers);
    L.prims = take(sizeof(Initializer) * o.n_primaries);
    L.vac = take(4 * n);
    uint64_t nvb = (n + kVacBlock - 1) / kVacBlock;
    L.vac_cnt = take(4 * nvb);
    L.init_cnt = take(4 * nvb);
    L.perm = take(4 * n);
    L.along_list = take(4 * n);
    L.lists = take(4ull * A_NUM * n);
    L.n_tiles = (uint32_t)((n + kSortTile - 1) / kSortTile);
    L.sort_cnt = take(4ull * 128 * L.n_tiles);
    L.bin_off = take(4 * 256);
    L.ctr = take(sizeof(Counters));
    uint64_t ntab = (uint64_t)o.max_materials * kTabPerMat * kNodes;
    L.tables64 = take(8 * ntab);
    L.tables32 = take(4 * ntab);
    L.mats = take(sizeof(MatDev) * o.max_materials);
    L.zp = take(8 * ((uint64_t)o.max_slabs + 1));
    L.smat = take(4 * (uint64_t)o.max_slabs);
    L.row_event = take(8 * (uint64_t)o.max_events);
    // deposit tallies in copies (page-padded): about one tally address per
    // track slot, at most 64 copies and 64 MiB.  Many events over many slabs
    // spread their deposits by themselves (one copy); a few large events put
    // thousands of tracks on each of their slabs
    L.edep_rs = align_up((uint64_t)o.max_events * o.max_slabs, 512);   // 512 x 8 B = 4 KiB
    L.n_rep_e = 1;
    while (L.n_rep_e < kMaxCounterCopies && 2ull * L.n_rep_e * o.max_events * o.max_slabs <= o.n_slots &&
           8ull * L.edep_rs * 2 * L.n_rep_e <= (64ull << 20))
        L.n_rep_e <<= 1;
    L.edep = take(8ull * L.edep_rs * L.n_rep_e);
    // per-event counters in copies (each copy's rows padded to whole 4 KiB
    // pages): one copy per 64 track slots per event row, at most 64 copies
    // and 64 MiB.  Many events share the slots' updates by themselves (one
    // copy for 10^4 events in 2^20 slots); a few large events put 10^5
    // tracks on each row
    L.ledger_rs = (uint32_t)align_up((uint64_t)o.max_events, 64);     // 64 x 72 B = 4.5 KiB
    L.live_rs = (uint32_t)align_up((uint64_t)o.max_events, 1024);     // 1024 x 4 B = 4 KiB
    L.n_rep = 1;
    while (L.n_rep < kMaxCounterCopies && 2ull * L.n_rep * o.max_events * 64 <= o.n_slots &&
           2ull * L.n_rep * (sizeof(Ledger) * L.ledger_rs + 4ull * L.live_rs) <= (64ull << 20))
        L.n_rep <<= 1;
    L.ledger = take(sizeof(Ledger) * (uint64_t)L.ledger_rs * L.n_rep);
    L.live = take(4ull * L.live_rs * L.n_rep);
    L.done_ring = take(8 * (uint64_t)o.max_events);
    L.row_gen = take(4 * (uint64_t)o.max_events);
    L.row_state = take(4 * (uint64_t)o.max_events);
    L.part_stride = (uint32_t)std::max<uint64_t>(2048, nvb);
    L.part = take(8ull * kNumW * L.part_stride);
    L.rowsum = take(8ull * kNumW);
    L.incr = take(8ull * o.max_materials * 2 * (kNodes - 1));
    L.drain_threads = (uint32_t)std::min<uint64_t>(kDrainThreadsMax, align_up(n, 256));
    L.drain_stack = take(sizeof(Initializer) * kDrainDepth * (uint64_t)L.drain_threads);
    L.regs = take(sizeof(RowReg) * kStagingCap);
    L.ledger_out = take(sizeof(Ledger) * (uint64_t)o.max_events);
    if (o.deterministic) {
        L.sec_cnt = take(n);
        L.sec_blk = take(4 * nvb);
        L.sec_rec = take(sizeof(Initializer) * 3 * n);
    }
    L.edep_out = take(8ull * o.max_events * o.max_slabs);
    L.x0 = take(8ull * o.max_materials);
    L.total = off;
    return L;
}

enum Role {
    R_VAC = 0, R_INIT, R_PRE /* reserved: the pre-step runs in the along-step kernels */, R_SORT, R_ALONG_NEUTRAL,
    R_ALONG_CHARGED, R_ALONG_FIELD,
    R_COMPTON, R_PHOTO, R_PAIR, R_MOLLER, R_BHABHA, R_BREMS, R_DRAIN, R_INTERACT_ALL, R_ANNIH, R_NUM
};
const char* kRoleNames[R_NUM] = {"vacancies", "init", "pre_step", "sort", "along_neutral", "along_charged",
                                 "along_field", "compton", "photoelectric", "pair", "moller", "bhabha",
                                 "bremsstrahlung", "drain", "interactions", "annihilation"};
static_assert(R_NUM <= 16, "the tuning block table holds 16 roles");

}  // namespace

struct ems_ctx {
    ems_options opt;
    Layout L;
    char* ws;
    hipStream_t stream;
    int device;
    // host mirrors
    uint32_t n_materials = 0, n_slabs = 0;
    bool have_mats = false, have_geom = false, have_tables = false;
    double ecut = 0.0, half_width = 0.0, B[3] = {0, 0, 0};
    std::vector<double> zp_host;   // z planes, for validating primaries
    double ln_e0, dlog;
    std::vector<ems_material> mats;
    // events
    std::unordered_map<uint64_t, uint32_t> row_of;
    std::vector<uint64_t> row_event;           // host copy, UINT64_MAX = free
    std::vector<uint32_t> free_rows;
    std::vector<uint64_t> row_pending;         // primaries pushed per row (for completion)
    std::vector<uint32_t> row_gen;             // bumped at every registration of a row
    // primaries ring
    uint64_t prim_end = 0;                     // host-owned
    uint32_t done_read = 0;                    // completion-ring entries already returned
    // pinned host memory
    Snapshot* snap = nullptr;                  // ring of snapshots
    int snap_slots = 4;
    hipEvent_t snap_ev[4];
    uint64_t snap_seq = 0;
    Initializer* staging = nullptr;            // pinned primary staging
    uint64_t staging_cap = 0;
    RowReg* reg_staging = nullptr;             // pinned staging of new row registrations (staging_cap entries)
    std::vector<RowReg> reg_pending;           // rows assigned on the host, not yet cleared on the device
    hipEvent_t staging_ev;
    bool staging_busy = false;
    // concurrent branches
    int n_streams = 1;
    hipStream_t workers[3] = {nullptr, nullptr, nullptr};
    hipEvent_t fork_ev[2];
    hipEvent_t join_ev[2][3];
    // graphs
    hipGraphExec_t graph = nullptr;
    int graph_iters = 0;
    int graph_no_init = -1;
    // tuning (switchable at run time)
    int policy = 0;
    uint32_t tail_threshold = 0;
    // resident-grid cache of the field along-step, per precision (FP64, FP32)
    // resident grids by kernel: [FP64, FP32] x [field along-step, both along-steps, fused interactions,
    // fused interactions with deterministic appends]
    int grid_bs[8] = {0};
    size_t grid_lds[8] = {0};
    uint32_t grid_resident[8] = {0};
    uint32_t phase_sort[2] = {0xFFFFFFFFu, 0xFFFFFFFFu};
    uint32_t drain_threshold = 0;   // ems_run drains below this many live + queued + pending tracks
    uint32_t drain_steps = kDrainStepsDefault;
    uint32_t reuse_parent = 0;        // parent-slot reuse for the first secondary
    uint32_t fuse_interactions = 0;   // one launch for the seven interaction kernels
    uint32_t fuse_along = 1;          // one launch for the photon and field along-steps
    int block[16] = {0};
    // profiling
    uint32_t prof_mask = 0;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> prof_events;
    double prof_ms[R_NUM] = {0};
    uint64_t prof_n[R_NUM] = {0};
    Snapshot last{};
};

namespace {

// The photon and field along-steps run as one launch: a field, one stream
// and the tuning's fuse_along.
bool fused_along(const ems_ctx* c)
{
    return c->fuse_along && c->n_streams == 1 && (c->B[0] != 0.0 || c->B[1] != 0.0 || c->B[2] != 0.0);
}

template <class R>
Dev<R> make_dev(const ems_ctx* c)
{
    Dev<R> d{};
    char* b = c->ws;
    const Layout& L = c->L;
    d.type = (uint8_t*)(b + L.type);
    d.action = (uint8_t*)(b + L.action);
    d.flags = (uint8_t*)(b + L.flags);
    d.nsearch = (uint8_t*)(b + L.nsearch);
    d.slab = (uint16_t*)(b + L.slab);
    d.row = (uint32_t*)(b + L.row);
    d.step = (uint32_t*)(b + L.step);
    // the 64-byte track records (x, y, z, key, then ux, uy, uz, T)
    char* rec = b + L.trk;
    d.x.base = d.y.base = d.z.base = d.key.base = rec;
    d.ux.base = d.uy.base = d.uz.base = d.T.base = rec;
    d.nl = (R*)(b + L.nl);
    d.xs = (R*)(b + L.xs);
    d.sphys = (double*)(b + L.sphys);
    d.sdone = (double*)(b + L.sdone);
    d.htry = (double*)(b + L.htry);
    d.n_slots = (uint32_t)c->opt.n_slots;
    d.queue = (Initializer*)(b + L.queue);
    d.queue_cap = c->opt.n_initializers;
    d.prims = (Initializer*)(b + L.prims);
    d.prim_cap = c->opt.n_primaries;
    d.vac = (uint32_t*)(b + L.vac);
    d.vac_cnt = (uint32_t*)(b + L.vac_cnt);
    d.init_cnt = (uint32_t*)(b + L.init_cnt);
    d.perm = (uint32_t*)(b + L.perm);
    d.lists = (uint32_t*)(b + L.lists);
    d.ctr = (Counters*)(b + L.ctr);
    d.tb.v = (const R*)(b + (sizeof(R) == 8 ? L.tables64 : L.tables32));
    d.tb.ln_e0 = (R)c->ln_e0;
    d.tb.dlog = (R)c->dlog;
    d.tb.inv_dlog = (R)(1.0 / c->dlog);
    d.zp = (const double*)(b + L.zp);
    d.smat = (const int32_t*)(b + L.smat);
    d.n_slabs = (int)c->n_slabs;
    d.W = c->half_width;
    d.B[0] = c->B[0]; d.B[1] = c->B[1]; d.B[2] = c->B[2];
    d.has_field = (c->B[0] != 0.0 || c->B[1] != 0.0 || c->B[2] != 0.0);
    d.ecut = c->ecut;
    d.seed = c->opt.seed;
    d.row_event = (const uint64_t*)(b + L.row_event);
    d.edep = (double*)(b + L.edep);
    d.ledger = (Ledger*)(b + L.ledger);
    d.edep_stride = (int)c->opt.max_slabs;
    d.edep_rep_mask = L.n_rep_e - 1;
    d.edep_rs = L.edep_rs;
    d.live = (unsigned int*)(b + L.live);
    d.rep_mask = L.n_rep - 1;
    d.ledger_rs = L.ledger_rs;
    d.live_rs = L.live_rs;
    d.done_ring = (unsigned long long*)(b + L.done_ring);
    d.row_gen = (const unsigned int*)(b + L.row_gen);
    d.row_state = (unsigned int*)(b + L.row_state);
    d.part = (unsigned long long*)(b + L.part);
    d.part_stride = L.part_stride;
    d.n_rows = c->opt.max_events;
    d.max_substeps = c->opt.max_substeps;
    d.sorted = c->policy == EMS_SORT_NONE ? 0 : 1;
    d.sorted2 = c->policy == EMS_SORT_NONE ? 0 : (c->policy == EMS_SORT_QUEUE ? 2 : 1);
    d.tail_threshold = c->tail_threshold;
    d.phase_sort1 = c->phase_sort[0];
    d.phase_sort2 = c->phase_sort[1];
    d.stage_tables = c->opt.lds_tables ? 1 : 0;
    d.reuse_parent = c->reuse_parent ? 1 : 0;
    d.msc = c->opt.msc ? 1 : 0;
    // deterministic appends keep the counted (ordered) partitioned fill
    d.fill_reserve = (c->opt.init_partition && !c->opt.deterministic) ? 1 : 0;
    d.det = c->opt.deterministic ? 1 : 0;
    d.along_list = (uint32_t*)(b + L.along_list);
    // the walk over listed slots is a reordering: not with the policy none
    d.compact_along = (c->policy != EMS_SORT_NONE && fused_along(c)) ? 1 : 0;
    d.sec_cnt = c->opt.deterministic ? (uint8_t*)(b + L.sec_cnt) : nullptr;
    d.sec_blk = c->opt.deterministic ? (uint32_t*)(b + L.sec_blk) : nullptr;
    d.sec_rec = c->opt.deterministic ? (Initializer*)(b + L.sec_rec) : nullptr;
    d.x0 = (const double*)(c->ws + c->L.x0);
    d.n_tab = (int)(c->n_materials * kTabPerMat * kNodes);
    return d;
}

__global__ void k_fill_u8(uint8_t* p, uint8_t v, uint64_t n)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_zero_bytes(uint8_t* p, uint64_t n)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

__global__ void k_set_prim_end(Counters* c, unsigned long long v) { c->prim_end = v; }

__global__ void k_reset_queue(Counters* c)
{
    c->queue_size = 0;
    c->overflow = 0;
}

// A batch of registrations {event, row, generation}: one block per row.
// Every copy of the row's ledger and live count is cleared.
__global__ void k_set_rows(const RowReg* regs, uint64_t* row_event, double* edep, Ledger* led, uint32_t n_slabs,
                           unsigned int* live, unsigned int* row_gen, unsigned int* row_state, uint32_t n_rep,
                           uint32_t ledger_rs, uint32_t live_rs, uint32_t n_rep_e, uint64_t edep_rs)
{
    const RowReg g = regs[blockIdx.x];
    for (uint32_t i = threadIdx.x; i < n_slabs * n_rep_e; i += blockDim.x)
        edep[(size_t)(i / n_slabs) * edep_rs + (size_t)g.row * n_slabs + i % n_slabs] = 0.0;
    for (uint32_t r = threadIdx.x; r < n_rep; r += blockDim.x) {
        led[(size_t)r * ledger_rs + g.row] = Ledger{};
        live[(size_t)r * live_rs + g.row] = 0u;
    }
    if (threadIdx.x == 0) {
        row_event[g.row] = g.ev;
        row_gen[g.row] = g.gen;
        row_state[g.row] = g.ev != UINT64_MAX ? 1u : 0u;
    }
}

// pushed primaries count toward their event until they retire (thread i
// adds to copy i mod n_rep of the live count)
__global__ void k_count_primaries(const Initializer* prims, uint64_t cap, uint64_t start, uint64_t n,
                                  unsigned int* live, uint32_t rep_mask, uint32_t live_rs)
{
    uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    atomicAdd(&live[(size_t)(i & rep_mask) * live_rs + prims[(start + i) % cap].row], 1u);
}

// Sum the copies of the deposit tallies of rows [row0, row0 + n) (stride
// n_slabs doubles) into out[0, n * n_slabs).
__global__ void k_edep_sum(const double* edep, uint32_t n_rep, uint64_t edep_rs, uint32_t n_slabs, uint32_t row0,
                           uint32_t n, double* out)
{
    const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (i >= (uint64_t)n * n_slabs) return;
    const uint64_t at = (uint64_t)row0 * n_slabs + i;
    double v = 0.0;
    for (uint32_t r = 0; r < n_rep; ++r) v += edep[r * edep_rs + at];
    out[i] = v;
}

// Sum the copies of the ledgers of rows [row0, row0 + n) into out[0, n).
__global__ void k_ledger_sum(const Ledger* led, uint32_t n_rep, uint32_t ledger_rs, uint32_t row0, uint32_t n,
                             Ledger* out)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Ledger s{};
    for (uint32_t r = 0; r < n_rep; ++r) {
        const Ledger& l = led[(size_t)r * ledger_rs + row0 + i];
        s.escaped += l.escaped;
        s.n_pair += l.n_pair;
        s.n_annih += l.n_annih;
        s.steps += l.steps;
        for (int t = 0; t < 3; ++t) s.n_sec[t] += l.n_sec[t];
        s.n_guard += l.n_guard;
        s.n_reject_cap += l.n_reject_cap;
    }
    out[i] = s;
}

// Sum each row of the per-block partial counters: block w sums row w.
__global__ void __launch_bounds__(256) k_sum_rows(const unsigned long long* part, uint32_t stride,
                                                  unsigned long long* rowsum)
{
    const unsigned long long* row = part + (size_t)blockIdx.x * stride;
    unsigned long long v = 0;
    for (uint32_t i = threadIdx.x; i < stride; i += blockDim.x) v += row[i];
    v = block_sum(v);
    if (threadIdx.x == 0) rowsum[blockIdx.x] = v;
}

// Copy the loop counters and the row sums of the partial counters
__global__ void k_snapshot(const Counters* c, const unsigned long long* acc, Snapshot* out)
{
    if (threadIdx.x == 0) {
        Snapshot s;
        s.queue_size = c->queue_size;
        s.prim_next = c->prim_next;
        s.prim_end = c->prim_end;
        s.iterations = c->iterations;
        unsigned long long steps = 0;
        for (int i = kStepsSlot; i < kNumW; ++i) steps += acc[i];
        s.steps_done = steps;
        s.n_vac = c->n_vac;
        s.n_alive = c->n_alive;
        s.overflow = c->overflow;
        s.done_count = c->done_count;
        for (int i = 0; i < kNumWork; ++i) s.work[i] = acc[i];
        *out = s;
    }
}

uint32_t grid_for(uint64_t n, int bs)
{
    uint64_t g = (n + bs - 1) / bs;
    const uint64_t cap = 256 * 8;   // 256 CUs x 8 resident blocks: grid-stride beyond that
    if (g > cap) g = cap;
    if (g == 0) g = 1;
    return (uint32_t)g;
}

// Launches the step kernels.  For a profiled role the role's first kernel
// carries the start event and its last kernel the stop event; both are
// stamped by the kernels' own dispatch packets (hipExtLaunchKernel), so the
// elapsed time is the execution of the role's kernels with no marker packets
// in between.
struct Launcher {
    ems_ctx* c;
    bool prof;
    hipEvent_t start = nullptr;
    template <class... KArgs, class... Args>
    void k(int role, bool first, bool last, void (*kernel)(KArgs...), dim3 g, dim3 b, size_t lds, hipStream_t st,
           Args... args)
    {
        if (!(prof && (c->prof_mask & (1u << role)))) {
            kernel<<<g, b, lds, st>>>(args...);
            return;
        }
        hipEvent_t a = nullptr, z = nullptr;
        if (first) {
            (void)hipEventCreate(&a);
            start = a;
        }
        if (last) (void)hipEventCreate(&z);
        hipExtLaunchKernelGGL(kernel, g, b, (uint32_t)lds, st, a, z, 0u, args...);
        if (last) {
            c->prof_events.push_back({role, {start, z}});
            start = nullptr;
        }
    }
    // a role made of one kernel
    template <class... KArgs, class... Args>
    void one(int role, void (*kernel)(KArgs...), dim3 g, dim3 b, size_t lds, hipStream_t st, Args... args)
    {
        k(role, true, true, kernel, g, b, lds, st, args...);
    }
};

// fork: workers [0, k) wait for the work enqueued so far on the main stream
void fork(ems_ctx* c, int point, int k)
{
    (void)hipEventRecord(c->fork_ev[point], c->stream);
    for (int i = 0; i < k; ++i) (void)hipStreamWaitEvent(c->workers[i], c->fork_ev[point], 0);
}

// join: the main stream waits for workers [0, k)
void join(ems_ctx* c, int point, int k)
{
    for (int i = 0; i < k; ++i) {
        (void)hipEventRecord(c->join_ev[point][i], c->workers[i]);
        (void)hipStreamWaitEvent(c->stream, c->join_ev[point][i], 0);
    }
}

// km: the key mode of the partition (0: next action; 2: the along-step
// action from the type, for the first sort); radix uses the matching 1 or 3
template <class R>
void launch_sort(ems_ctx* c, const Dev<R>& d, Launcher& ln, int km)
{
    const int policy = c->policy;
    uint32_t* cnt = (uint32_t*)(c->ws + c->L.sort_cnt);
    uint32_t* tot = (uint32_t*)(c->ws + c->L.bin_off);
    uint32_t nt = c->L.n_tiles;
    uint32_t n = d.n_slots;
    if (policy == EMS_SORT_PARTITION || policy == EMS_SORT_QUEUE) {
        ln.k(R_SORT, true, false, k_sort_hist<R, 16>, dim3(nt), dim3(kSortThreads), 0, c->stream, d, km,
             (const uint8_t*)nullptr, n, cnt, nt);
        ln.k(R_SORT, false, false, k_sort_scan<16>, dim3(16), dim3(256), 0, c->stream, cnt, nt, (const Counters*)d.ctr,
             tot, km >= 2 ? 1u : 2u);
        ln.k(R_SORT, false, true, k_sort_scatter<R, 16>, dim3(nt), dim3(kSortThreads), 0, c->stream, d, km,
             (const uint8_t*)nullptr, n, (const uint32_t*)cnt, nt, (const uint32_t*)tot, d.perm);
    } else {
        const int km1 = km == 2 ? 3 : 1;
        ln.k(R_SORT, true, false, k_sort_hist<R, 128>, dim3(nt), dim3(kSortThreads), 0, c->stream, d, km1,
             (const uint8_t*)nullptr, n, cnt, nt);
        ln.k(R_SORT, false, false, k_sort_scan<128>, dim3(128), dim3(256), 0, c->stream, cnt, nt,
             (const Counters*)d.ctr, tot, km1 >= 2 ? 1u : 2u);
        ln.k(R_SORT, false, true, k_sort_scatter<R, 128>, dim3(nt), dim3(kSortThreads), 0, c->stream, d, km1,
             (const uint8_t*)nullptr, n, (const uint32_t*)cnt, nt, (const uint32_t*)tot, d.perm);
    }
}

// The blocks of `kern` the device holds at once (cached per kernel slot k
// and launch shape), at most g.
uint32_t resident_grid(ems_ctx* c, const void* kern, int k, uint32_t g, int bs, size_t lds)
{
    if (c->grid_bs[k] != bs || c->grid_lds[k] != lds) {
        int nb = 0, cus = 0, dev = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
            cus = 256;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, bs, lds) != hipSuccess || nb < 1)
            nb = 1;
        c->grid_resident[k] = (uint32_t)(nb * cus);
        c->grid_bs[k] = bs;
        c->grid_lds[k] = lds;
    }
    return c->grid_resident[k] < g ? c->grid_resident[k] : g;
}

// Grid of the field (or both) along-steps with a sort policy: one resident
// round (each thread then walks its tracks at the grid stride with the next
// track's loads in flight), at most the slot-covering grid.  Measured: one
// resident round 2.97e9 track-steps/s, two 2.90e9, the slot-covering grid
// (one track per thread) 2.84e9.
template <class R>
uint32_t field_grid(ems_ctx* c, uint32_t g, int bs, size_t lds, bool both)
{
    const void* kern = both ? reinterpret_cast<const void*>(k_along_both<R>)
                            : reinterpret_cast<const void*>(k_along_field<R>);
    return resident_grid(c, kern, (sizeof(R) == 8 ? 0 : 1) + (both ? 2 : 0), g, bs, lds);
}

// The interaction kernels of an iteration: one fused launch, or seven on
// the library's streams.
template <class R, bool DET>
void launch_interactions(ems_ctx* c, const Dev<R>& d, Launcher& ln, int nw)
{
    const int bs_def = c->opt.block_size > 0 ? c->opt.block_size : 256;
    const uint32_t n = d.n_slots;
    auto B = [&](int role) { return c->block[role] > 0 ? c->block[role] : bs_def; };
    auto G = [&](int role) { return grid_for(n, B(role)); };
    hipStream_t st = c->stream;
    if (c->fuse_interactions) {
        // all seven actions in one launch over the combined index range
        // one resident round of blocks walks the combined range (the slot
        // covering grid would launch thousands of blocks that find nothing)
        const uint32_t g = resident_grid(c, reinterpret_cast<const void*>(k_interact_all<R, DET>),
                                         4 + (sizeof(R) == 8 ? 0 : 1) + (DET ? 2 : 0), G(R_INTERACT_ALL),
                                         B(R_INTERACT_ALL), 0);
        ln.one(R_INTERACT_ALL, k_interact_all<R, DET>, dim3(g), dim3(B(R_INTERACT_ALL)), 0, st, d);
        return;
    }
    // seven independent branches spread over the streams
    if (nw > 0) fork(c, 1, nw);
    auto on = [&](int k) { return k % c->n_streams == 0 ? st : c->workers[k % c->n_streams - 1]; };
    ln.one(R_COMPTON, k_interact<R, P_COMPTON, DET>, dim3(G(R_COMPTON)), dim3(B(R_COMPTON)), 0, on(0), d);
    ln.one(R_PHOTO, k_interact<R, P_PHOTO, DET>, dim3(G(R_PHOTO)), dim3(B(R_PHOTO)), 0, on(1), d);
    ln.one(R_PAIR, k_interact<R, P_PAIR, DET>, dim3(G(R_PAIR)), dim3(B(R_PAIR)), 0, on(2), d);
    ln.one(R_MOLLER, k_interact<R, P_MOLLER, DET>, dim3(G(R_MOLLER)), dim3(B(R_MOLLER)), 0, on(3), d);
    ln.one(R_BHABHA, k_interact<R, P_BHABHA, DET>, dim3(G(R_BHABHA)), dim3(B(R_BHABHA)), 0, on(4), d);
    ln.one(R_BREMS, k_interact<R, P_BREMS, DET>, dim3(G(R_BREMS)), dim3(B(R_BREMS)), 0, on(5), d);
    ln.one(R_ANNIH, k_interact<R, P_ANNIH, DET>, dim3(G(R_ANNIH)), dim3(B(R_ANNIH)), 0, on(6), d);
    if (nw > 0) join(c, 1, nw);
}

template <class R>
void launch_iteration(ems_ctx* c, bool no_init, bool prof)
{
    Dev<R> d = make_dev<R>(c);
    Launcher ln{c, prof};
    const int bs_def = c->opt.block_size > 0 ? c->opt.block_size : 256;
    const uint32_t n = d.n_slots;
    const uint32_t nvb = (n + kVacBlock - 1) / kVacBlock;
    const uint32_t nvs = (n + kVacSpan - 1) / kVacSpan;      // vacancy blocks
    auto B = [&](int role) { return c->block[role] > 0 ? c->block[role] : bs_def; };
    auto G = [&](int role) { return grid_for(n, B(role)); };
    hipStream_t st = c->stream;
    ln.k(R_VAC, true, false, k_vac_count<R>, dim3(nvs), dim3(kVacBlock), 0, st, d);
    ln.k(R_VAC, false, true, k_vac_scatter<R>, dim3(nvs), dim3(kVacBlock), 0, st, d, no_init ? 0 : 1,
         d.compact_along ? d.along_list : (uint32_t*)nullptr);
    if (!no_init) {
        if (d.fill_reserve) {
            ln.one(R_INIT, k_init_reserve<R>, dim3(nvb), dim3(kVacBlock), 0, st, d);
        } else if (c->opt.init_partition) {
            ln.k(R_INIT, true, false, k_init_count<R>, dim3(nvb), dim3(kVacBlock), 0, st, d);
            ln.k(R_INIT, false, true, k_init<R, true>, dim3(nvb), dim3(kVacBlock), 0, st, d);
        } else {
            ln.one(R_INIT, k_init<R, false>, dim3(nvb), dim3(kVacBlock), 0, st, d);
        }
    }
    const size_t lds = d.stage_tables ? (size_t)d.n_tab * sizeof(R) : 0;
    // (the along-step kernels run the pre-step of their tracks)
    // a sort point whose phase mask is empty never reorders: its kernels are
    // not launched at all (not even to return at once)
    if (d.sorted == 1 && c->phase_sort[0] != 0u) launch_sort<R>(c, d, ln, 2);
    // along-step: photons and leptons are independent branches, or one
    // launch for both in a field on one stream (tuning fuse_along)
    const int nw = c->n_streams - 1;
    if (fused_along(c)) {
        ln.one(R_ALONG_FIELD, k_along_both<R>,
               dim3(c->policy == EMS_SORT_NONE ? G(R_ALONG_FIELD)
                                               : field_grid<R>(c, G(R_ALONG_FIELD), B(R_ALONG_FIELD), lds, true)),
               dim3(B(R_ALONG_FIELD)), lds, st, d);
    } else {
        hipStream_t s_neutral = nw > 0 ? c->workers[0] : st;
        if (nw > 0) fork(c, 0, 1);
        ln.one(R_ALONG_NEUTRAL, k_along_straight<R, false>, dim3(G(R_ALONG_NEUTRAL)), dim3(B(R_ALONG_NEUTRAL)), lds,
               s_neutral, d);
        if (d.has_field)
            ln.one(R_ALONG_FIELD, k_along_field<R>,
                   dim3(c->policy == EMS_SORT_NONE ? G(R_ALONG_FIELD)
                                                   : field_grid<R>(c, G(R_ALONG_FIELD), B(R_ALONG_FIELD), lds, false)),
                   dim3(B(R_ALONG_FIELD)), lds, st, d);
        else
            ln.one(R_ALONG_CHARGED, k_along_straight<R, true>, dim3(G(R_ALONG_CHARGED)), dim3(B(R_ALONG_CHARGED)),
                   lds, st, d);
        if (nw > 0) join(c, 0, 1);
    }
    if (d.sorted2 == 1 && c->phase_sort[1] != 0u) launch_sort<R>(c, d, ln, 0);
    if (d.det) launch_interactions<R, true>(c, d, ln, nw);
    else launch_interactions<R, false>(c, d, ln, nw);
    if (d.det) {
        // deterministic appends: the staged secondaries in interaction order
        ln.k(R_INIT, true, false, k_sec_count<R>, dim3(nvb), dim3(kVacBlock), 0, st, d);
        ln.k(R_INIT, false, true, k_sec_scatter<R>, dim3(nvb), dim3(kVacBlock), 0, st, d);
    }
}

void launch_iteration_any(ems_ctx* c, bool no_init, bool prof)
{
    if (c->opt.precision == EMS_MIXED) launch_iteration<float>(c, no_init, prof);
    else launch_iteration<double>(c, no_init, prof);
}

// One drain iteration: vacancies (and the list of occupied slots), fill from
// the initializer buffer and the pending primaries, then one drain launch in
// which every block steps its share of the slots in rounds.
template <class R>
void launch_drain(ems_ctx* c, uint32_t threads)
{
    Dev<R> d = make_dev<R>(c);
    Launcher ln{c, c->prof_mask != 0};
    const uint32_t n = d.n_slots;
    const uint32_t nvb = (n + kVacBlock - 1) / kVacBlock;
    const uint32_t nvs = (n + kVacSpan - 1) / kVacSpan;      // vacancy blocks
    hipStream_t st = c->stream;
    uint32_t* live_list = (uint32_t*)(c->ws + c->L.perm);
    ln.k(R_VAC, true, false, k_vac_count<R>, dim3(nvs), dim3(kVacBlock), 0, st, d);
    ln.k(R_VAC, false, true, k_vac_scatter<R>, dim3(nvs), dim3(kVacBlock), 0, st, d, 1, live_list);
    ln.one(R_INIT, k_init<R, false>, dim3(nvb), dim3(kVacBlock), 0, st, d);
    const size_t lds = d.stage_tables ? (size_t)d.n_tab * sizeof(R) : 0;
    ln.one(R_DRAIN, k_drain<R>, dim3((threads + 255) / 256), dim3(256), lds, st, d, (const uint32_t*)live_list,
           (Initializer*)(c->ws + c->L.drain_stack), threads, kDrainDepth, c->drain_steps);
}

void launch_drain_any(ems_ctx* c, uint32_t threads)
{
    if (c->opt.precision == EMS_MIXED) launch_drain<float>(c, threads);
    else launch_drain<double>(c, threads);
}

// Record the events whose rows emptied in the iterations launched so far.
// The host reads completions only between launch groups, so one scan after
// each group (graph batch, iteration loop or drain launch) finds exactly what
// a scan after every iteration would.
void launch_completions(ems_ctx* c)
{
    const uint32_t nb = (c->opt.max_events + 255) / 256;
    if (c->opt.precision == EMS_MIXED)
        hipLaunchKernelGGL((k_scan_completions<float>), dim3(nb), dim3(256), 0, c->stream, make_dev<float>(c));
    else
        hipLaunchKernelGGL((k_scan_completions<double>), dim3(nb), dim3(256), 0, c->stream, make_dev<double>(c));
}

// ---- fixed scratch for the allocation-free sort entry point --------------------
// The per-tile histograms and bin totals of one sort of up to kNoAllocMaxKeys
// keys with up to 128 bins: 128 * 8192 + 128 words = 4 MiB + 512 B, held by
// every device the library runs on until the process ends.  Host code never
// uses the array's name as an address: each device's copy has its own
// address, taken once per device with hipGetSymbolAddress.
constexpr uint64_t kNoAllocMaxKeys = 1ull << 23;
constexpr uint64_t kNoAllocTiles = kNoAllocMaxKeys / kSortTile;
constexpr uint64_t kNoAllocWords = 128 * kNoAllocTiles + 128;
__device__ __align__(256) uint32_t scratch[kNoAllocWords];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint32_t* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (taken on first use per
// device, with that device current).  Returns null with the error set.
uint32_t* scratch_on_device(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) {
        fail(EMS_ERR_DEVICE, "device index beyond the scratch table");
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            fail(EMS_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            return nullptr;
        }
        g_scratch_ptr[dev] = (uint32_t*)ptr;
    }
    return g_scratch_ptr[dev];
}

ems_status check_ready(ems_ctx* c)
{
    if (!c) return fail(EMS_ERR_INVALID_ARG, "null context");
    if (!c->have_geom || !c->have_tables || !c->have_mats)
        return fail(EMS_ERR_STATE, "materials, geometry and tables must be loaded first");
    return EMS_OK;
}

ems_status drop_graph(ems_ctx* c)
{
    if (c->graph) {
        HIP_TRY(hipGraphExecDestroy(c->graph));
        c->graph = nullptr;
    }
    return EMS_OK;
}

// launch `iters` iterations, through a captured graph when configured
ems_status launch_batch(ems_ctx* c, int iters, bool no_init)
{
    bool prof = c->prof_mask != 0;
    int gi = c->opt.graph_iterations;
    if (gi > 0 && !prof && iters == gi) {
        if (c->stream == nullptr) return fail(EMS_ERR_INVALID_ARG, "graph capture needs a non-null stream");
        if (!c->graph || c->graph_iters != gi || c->graph_no_init != (int)no_init) {
            ems_status s = drop_graph(c);
            if (s != EMS_OK) return s;
            hipGraph_t g;
            HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
            for (int i = 0; i < gi; ++i) launch_iteration_any(c, no_init, false);
            launch_completions(c);
            HIP_TRY(hipStreamEndCapture(c->stream, &g));
            HIP_TRY(hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0));
            HIP_TRY(hipGraphDestroy(g));
            c->graph_iters = gi;
            c->graph_no_init = (int)no_init;
        }
        HIP_TRY(hipGraphLaunch(c->graph, c->stream));
    } else {
        for (int i = 0; i < iters; ++i) launch_iteration_any(c, no_init, prof);
        launch_completions(c);
        HIP_TRY(hipGetLastError());
    }
    return EMS_OK;
}

// counters snapshot into `out` (device-visible pinned memory), on the stream
void launch_snapshot(ems_ctx* c, Snapshot* out)
{
    unsigned long long* rowsum = (unsigned long long*)(c->ws + c->L.rowsum);
    hipLaunchKernelGGL(k_sum_rows, dim3(kNumW), dim3(256), 0, c->stream,
                       (const unsigned long long*)(c->ws + c->L.part), c->L.part_stride, rowsum);
    hipLaunchKernelGGL(k_snapshot, dim3(1), dim3(64), 0, c->stream, (const Counters*)(c->ws + c->L.ctr),
                       (const unsigned long long*)rowsum, out);
}

ems_status snapshot_now(ems_ctx* c, Snapshot* out)
{
    Snapshot* slot = &c->snap[0];
    launch_snapshot(c, slot);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(c->stream));
    *out = *slot;
    c->last = *out;
    return EMS_OK;
}

void to_counters(const Snapshot& s, ems_counters* out)
{
    out->iterations = s.iterations;
    out->alive = s.n_alive;
    out->queued = s.queue_size;
    out->pending_primaries = s.prim_end - s.prim_next;
    out->steps = s.steps_done;
    out->overflow = s.overflow;
    out->completed = s.done_count;
    for (int i = 0; i < kNumWork; ++i) out->work[i] = s.work[i];
}

template <class R>
__global__ void k_inject(Dev<R> d, const ems_track* t, uint64_t n)
{
    uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (i >= d.n_slots) return;
    if (i >= n || t[i].type < 0) {
        d.type[i] = kDead;
        d.action[i] = A_NONE;
        return;
    }
    const ems_track& r = t[i];
    atomicAdd(live_of(d, r.row), 1u);
    d.type[i] = (uint8_t)r.type;
    d.action[i] = A_IDLE;
    d.flags[i] = 0;
    d.nsearch[i] = 0;
    d.slab[i] = (uint16_t)r.slab;
    d.row[i] = r.row;
    d.step[i] = r.step;
    d.key[i] = r.key;
    d.T[i] = (R)r.T;
    d.nl[i] = (R)r.nl;
    d.xs[i] = R(0);
    d.sphys[i] = 0.0;
    d.sdone[i] = 0.0;
    d.htry[i] = 0.0;
    d.x[i] = r.r[0]; d.y[i] = r.r[1]; d.z[i] = r.r[2];
    d.ux[i] = (R)r.u[0]; d.uy[i] = (R)r.u[1]; d.uz[i] = (R)r.u[2];
}

template <class R>
__global__ void k_read_tracks(Dev<R> d, ems_track* t, uint64_t n)
{
    uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    ems_track& r = t[i];
    r.key = d.key[i];
    r.row = d.row[i];
    r.step = d.step[i];
    r.type = d.type[i] == kDead ? -1 : (int32_t)d.type[i];
    r.slab = d.slab[i];
    r.T = (double)d.T[i];
    r.nl = (double)d.nl[i];
    r.r[0] = d.x[i]; r.r[1] = d.y[i]; r.r[2] = d.z[i];
    r.u[0] = (double)d.ux[i]; r.u[1] = (double)d.uy[i]; r.u[2] = (double)d.uz[i];
}

__global__ void k_read_queue(const Initializer* q, uint64_t n, ems_track* t)
{
    uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Initializer& a = q[i];
    ems_track& r = t[i];
    r.key = a.key;
    r.row = a.row;
    r.step = 0;
    r.type = a.type;
    r.slab = a.slab;
    r.T = a.T;
    r.nl = -1.0;
    r.r[0] = a.r[0]; r.r[1] = a.r[1]; r.r[2] = a.r[2];
    r.u[0] = a.u[0]; r.u[1] = a.u[1]; r.u[2] = a.u[2];
}

ems_status assign_row(ems_ctx* c, uint64_t ev, uint32_t* row)
{
    auto it = c->row_of.find(ev);
    if (it != c->row_of.end()) {
        *row = it->second;
        return EMS_OK;
    }
    if (c->free_rows.empty()) return fail(EMS_ERR_CAPACITY, "no free event row (max_events)");
    uint32_t r = c->free_rows.back();
    c->free_rows.pop_back();
    c->row_of[ev] = r;
    c->row_event[r] = ev;
    c->row_gen[r] += 1;
    c->reg_pending.push_back(RowReg{ev, r, c->row_gen[r]});
    *row = r;
    return EMS_OK;
}

// Clear and register on the device the rows assigned since the last flush
// (one kernel); the caller guarantees the registration staging is free.
ems_status flush_rows(ems_ctx* c)
{
    size_t done = 0;
    while (done < c->reg_pending.size()) {
        size_t k = std::min<size_t>(c->reg_pending.size() - done, c->staging_cap);
        if (c->staging_busy) {
            HIP_TRY(hipEventSynchronize(c->staging_ev));
            c->staging_busy = false;
        }
        std::memcpy(c->reg_staging, c->reg_pending.data() + done, sizeof(RowReg) * k);
        RowReg* dev = (RowReg*)(c->ws + c->L.regs);
        HIP_TRY(hipMemcpyAsync(dev, c->reg_staging, sizeof(RowReg) * k, hipMemcpyHostToDevice, c->stream));
        hipLaunchKernelGGL(k_set_rows, dim3((uint32_t)k), dim3(256), 0, c->stream, (const RowReg*)dev,
                           (uint64_t*)(c->ws + c->L.row_event), (double*)(c->ws + c->L.edep),
                           (Ledger*)(c->ws + c->L.ledger), (uint32_t)c->opt.max_slabs,
                           (unsigned int*)(c->ws + c->L.live), (unsigned int*)(c->ws + c->L.row_gen),
                           (unsigned int*)(c->ws + c->L.row_state), c->L.n_rep, c->L.ledger_rs, c->L.live_rs,
                           c->L.n_rep_e, c->L.edep_rs);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipEventRecord(c->staging_ev, c->stream));
        c->staging_busy = true;
        done += k;
    }
    c->reg_pending.clear();
    return EMS_OK;
}

}  // namespace

// =============================================================================== ABI
extern "C" {

uint32_t ems_abi_version(void) { return EMS_ABI_VERSION; }

const char* ems_last_error(void) { return g_err.c_str(); }

static ems_status validate(const ems_options* o)
{
    if (!o) return fail(EMS_ERR_INVALID_ARG, "null options");
    if (o->abi_version != EMS_ABI_VERSION) return fail(EMS_ERR_INVALID_ARG, "abi_version mismatch");
    if (o->precision != EMS_FP64 && o->precision != EMS_MIXED) return fail(EMS_ERR_INVALID_ARG, "precision");
    if (o->n_slots == 0 || o->n_slots > (1ull << 30)) return fail(EMS_ERR_INVALID_ARG, "n_slots must be in [1, 2^30]");
    if (o->n_initializers == 0 || o->n_primaries == 0) return fail(EMS_ERR_INVALID_ARG, "buffer capacities");
    if (o->max_events == 0 || o->max_slabs == 0 || o->max_slabs > 65534 || o->max_materials == 0)
        return fail(EMS_ERR_INVALID_ARG, "max_events / max_slabs / max_materials");
    if (o->sort_policy < 0 || o->sort_policy > 3) return fail(EMS_ERR_INVALID_ARG, "sort_policy");
    int bs = o->block_size;
    if (bs != 0 && (bs < 64 || bs > 512 || (bs % 64) != 0)) return fail(EMS_ERR_INVALID_ARG, "block_size");
    if (o->graph_iterations < 0) return fail(EMS_ERR_INVALID_ARG, "graph_iterations");
    if (o->streams < 0 || o->streams > 4) return fail(EMS_ERR_INVALID_ARG, "streams must be in [0, 4]");
    if (o->msc != 0 && o->msc != 1) return fail(EMS_ERR_INVALID_ARG, "msc must be 0 or 1");
    if (o->deterministic != 0 && o->deterministic != 1) return fail(EMS_ERR_INVALID_ARG, "deterministic must be 0 or 1");
    if (o->deterministic && o->sort_policy == EMS_SORT_QUEUE)
        return fail(EMS_ERR_INVALID_ARG, "deterministic appends do not combine with the queue policy");
    return EMS_OK;
}

ems_status ems_query_workspace(const ems_options* opt, uint64_t* bytes)
{
    ems_status s = validate(opt);
    if (s != EMS_OK) return s;
    if (!bytes) return fail(EMS_ERR_INVALID_ARG, "null bytes");
    *bytes = make_layout(*opt).total;
    return EMS_OK;
}

ems_status ems_create(const ems_options* opt, void* device_workspace, uint64_t bytes, void* hip_stream, ems_ctx** out)
{
    ems_status s = validate(opt);
    if (s != EMS_OK) return s;
    if (!device_workspace || !out) return fail(EMS_ERR_INVALID_ARG, "null workspace or out");
    if (((uintptr_t)device_workspace & 255) != 0) return fail(EMS_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    Layout L = make_layout(*opt);
    if (bytes < L.total) return fail(EMS_ERR_INVALID_ARG, "workspace too small");
    ems_ctx* c = new ems_ctx();
    c->opt = *opt;
    c->L = L;
    c->ws = (char*)device_workspace;
    c->stream = (hipStream_t)hip_stream;
    c->ln_e0 = std::log(kEmin);
    c->dlog = std::log(10.0) / 20.0;
    (void)hipGetDevice(&c->device);
    if (!scratch_on_device(c->device)) {
        delete c;
        return EMS_ERR_DEVICE;
    }
    c->row_event.assign(opt->max_events, UINT64_MAX);
    c->row_pending.assign(opt->max_events, 0);
    c->row_gen.assign(opt->max_events, 0);
    for (uint32_t r = opt->max_events; r > 0; --r) c->free_rows.push_back(r - 1);
    auto cleanup = [&](ems_status st) { ems_destroy(c); return st; };
    if (hipHostMalloc((void**)&c->snap, sizeof(Snapshot) * c->snap_slots, hipHostMallocDefault) != hipSuccess)
        return cleanup(fail(EMS_ERR_DEVICE, "hipHostMalloc snapshot"));
    for (int i = 0; i < c->snap_slots; ++i) (void)hipEventCreateWithFlags(&c->snap_ev[i], hipEventDisableTiming);
    c->staging_cap = kStagingCap;
    if (hipHostMalloc((void**)&c->staging, sizeof(Initializer) * c->staging_cap, hipHostMallocDefault) != hipSuccess)
        return cleanup(fail(EMS_ERR_DEVICE, "hipHostMalloc staging"));
    if (hipHostMalloc((void**)&c->reg_staging, sizeof(RowReg) * c->staging_cap, hipHostMallocDefault) != hipSuccess)
        return cleanup(fail(EMS_ERR_DEVICE, "hipHostMalloc registration staging"));
    (void)hipEventCreateWithFlags(&c->staging_ev, hipEventDisableTiming);
    c->policy = opt->sort_policy;
    c->n_streams = opt->streams > 1 ? opt->streams : 1;
    for (int i = 0; i < c->n_streams - 1; ++i)
        if (hipStreamCreateWithFlags(&c->workers[i], hipStreamNonBlocking) != hipSuccess)
            return cleanup(fail(EMS_ERR_DEVICE, "hipStreamCreate"));
    for (int p = 0; p < 2; ++p) {
        (void)hipEventCreateWithFlags(&c->fork_ev[p], hipEventDisableTiming);
        for (int i = 0; i < 3; ++i) (void)hipEventCreateWithFlags(&c->join_ev[p][i], hipEventDisableTiming);
    }
    // clear state: all slots vacant, counters and tallies zero, rows unassigned
    uint64_t n = opt->n_slots;
    hipLaunchKernelGGL(k_fill_u8, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, (uint8_t*)(c->ws + L.type), kDead, n);
    hipLaunchKernelGGL(k_fill_u8, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, (uint8_t*)(c->ws + L.action), A_NONE, n);
    hipLaunchKernelGGL(k_zero_bytes, dim3(1), dim3(256), 0, c->stream, (uint8_t*)(c->ws + L.ctr), (uint64_t)sizeof(Counters));
    uint64_t tb = L.incr - L.row_event;   // row_event, edep, ledger are contiguous
    hipLaunchKernelGGL(k_fill_u8, dim3(grid_for(8ull * opt->max_events, 256)), dim3(256), 0, c->stream,
                       (uint8_t*)(c->ws + L.row_event), (uint8_t)0xFF, 8ull * opt->max_events);
    hipLaunchKernelGGL(k_zero_bytes, dim3(grid_for(tb, 256)), dim3(256), 0, c->stream, (uint8_t*)(c->ws + L.edep),
                       L.incr - L.edep);
    if (opt->deterministic)
        hipLaunchKernelGGL(k_zero_bytes, dim3(grid_for(n, 256)), dim3(256), 0, c->stream,
                           (uint8_t*)(c->ws + L.sec_cnt), n);
    if (hipGetLastError() != hipSuccess) return cleanup(fail(EMS_ERR_DEVICE, "initial clear failed"));
    *out = c;
    return EMS_OK;
}

void ems_destroy(ems_ctx* c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    if (c->graph) (void)hipGraphExecDestroy(c->graph);
    for (auto& e : c->prof_events) {
        (void)hipEventDestroy(e.second.first);
        (void)hipEventDestroy(e.second.second);
    }
    if (c->snap) {
        (void)hipHostFree(c->snap);
        for (int i = 0; i < c->snap_slots; ++i) (void)hipEventDestroy(c->snap_ev[i]);
    }
    if (c->reg_staging) (void)hipHostFree(c->reg_staging);
    if (c->staging) {
        (void)hipHostFree(c->staging);
        (void)hipEventDestroy(c->staging_ev);
        for (int i = 0; i < 3; ++i)
            if (c->workers[i]) (void)hipStreamDestroy(c->workers[i]);
        for (int p = 0; p < 2; ++p) {
            (void)hipEventDestroy(c->fork_ev[p]);
            for (int i = 0; i < 3; ++i) (void)hipEventDestroy(c->join_ev[p][i]);
        }
    }
    delete c;
}

ems_status ems_load_materials(ems_ctx* c, const ems_material* m, uint32_t n)
{
    if (!c || !m || n == 0) return fail(EMS_ERR_INVALID_ARG, "null or empty materials");
    if (n > c->opt.max_materials) return fail(EMS_ERR_CAPACITY, "too many materials");
    std::vector<MatDev> md(n);
    for (uint32_t i = 0; i < n; ++i) {
        if (!(m[i].Z > 0 && m[i].A > 0 && m[i].density > 0 && m[i].I_eV > 0))
            return fail(EMS_ERR_INVALID_ARG, "material values must be positive");
        md[i] = MatDev{m[i].Z, m[i].A, m[i].density, m[i].I_eV};
    }
    HIP_TRY(hipMemcpyAsync(c->ws + c->L.mats, md.data(), sizeof(MatDev) * n, hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(k_material_x0, dim3((n + 63) / 64), dim3(64), 0, c->stream,
                       (const MatDev*)(c->ws + c->L.mats), (int)n, (double*)(c->ws + c->L.x0));
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->mats.assign(m, m + n);
    c->n_materials = n;
    c->have_mats = true;
    c->have_tables = false;
    return drop_graph(c);
}

ems_status ems_load_geometry(ems_ctx* c, const double* zp, const int32_t* sm, uint32_t n_slabs, double half_width,
                             const double B[3])
{
    if (!c || !zp || !sm || !B || n_slabs == 0) return fail(EMS_ERR_INVALID_ARG, "null geometry");
    if (n_slabs > c->opt.max_slabs) return fail(EMS_ERR_CAPACITY, "too many slabs");
    if (!c->have_mats) return fail(EMS_ERR_STATE, "load materials first");
    for (uint32_t i = 0; i < n_slabs; ++i) {
        if (!(zp[i + 1] > zp[i])) return fail(EMS_ERR_INVALID_ARG, "z planes must increase");
        if (sm[i] < 0 || (uint32_t)sm[i] >= c->n_materials) return fail(EMS_ERR_INVALID_ARG, "slab material index");
    }
    if (!(half_width > 0)) return fail(EMS_ERR_INVALID_ARG, "half_width");
    HIP_TRY(hipMemcpyAsync(c->ws + c->L.zp, zp, 8ull * (n_slabs + 1), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->ws + c->L.smat, sm, 4ull * n_slabs, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->n_slabs = n_slabs;
    c->half_width = half_width;
    c->zp_host.assign(zp, zp + n_slabs + 1);
    c->B[0] = B[0]; c->B[1] = B[1]; c->B[2] = B[2];
    c->have_geom = true;
    return drop_graph(c);
}

static ems_status finish_tables(ems_ctx* c, double ecut)
{
    uint64_t ntab = (uint64_t)c->n_materials * kTabPerMat * kNodes;
    hipLaunchKernelGGL(k_tables_to_f32, dim3((ntab + 255) / 256), dim3(256), 0, c->stream,
                       (const double*)(c->ws + c->L.tables64), (float*)(c->ws + c->L.tables32), (int)ntab);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->ecut = ecut;
    c->have_tables = true;
    return drop_graph(c);
}

ems_status ems_build_tables(ems_ctx* c, double ecut)
{
    if (!c) return fail(EMS_ERR_INVALID_ARG, "null context");
    if (!c->have_mats) return fail(EMS_ERR_STATE, "load materials first");
    if (!(ecut > kEmin && ecut < 1.0e5)) return fail(EMS_ERR_INVALID_ARG, "cut outside the table range");
    int nm = (int)c->n_materials;
    const MatDev* md = (const MatDev*)(c->ws + c->L.mats);
    double* t64 = (double*)(c->ws + c->L.tables64);
    double* incr = (double*)(c->ws + c->L.incr);
    hipLaunchKernelGGL(k_build_xs, dim3((nm * kNodes + 127) / 128), dim3(128), 0, c->stream, md, nm, ecut, c->ln_e0,
                       c->dlog, t64);
    hipLaunchKernelGGL(k_range_increments, dim3((nm * 2 * (kNodes - 1) + 127) / 128), dim3(128), 0, c->stream, md, nm,
                       ecut, c->ln_e0, c->dlog, incr);
    hipLaunchKernelGGL(k_range_accumulate, dim3(1), dim3(64), 0, c->stream, md, nm, ecut, c->ln_e0,
                       (const double*)incr, t64);
    HIP_TRY(hipGetLastError());
    return finish_tables(c, ecut);
}

ems_status ems_load_tables(ems_ctx* c, const double* tables, uint32_t n_materials, double ecut)
{
    if (!c || !tables) return fail(EMS_ERR_INVALID_ARG, "null tables");
    if (!c->have_mats || n_materials != c->n_materials) return fail(EMS_ERR_STATE, "tables must match loaded materials");
    if (!(ecut > kEmin && ecut < 1.0e5)) return fail(EMS_ERR_INVALID_ARG, "cut outside the table range");
    HIP_TRY(hipMemcpyAsync(c->ws + c->L.tables64, tables, 8ull * n_materials * kTabPerMat * kNodes,
                           hipMemcpyHostToDevice, c->stream));
    return finish_tables(c, ecut);
}

ems_status ems_read_tables(ems_ctx* c, double* out, uint64_t n_doubles)
{
    if (!c || !out) return fail(EMS_ERR_INVALID_ARG, "null");
    if (!c->have_tables) return fail(EMS_ERR_STATE, "no tables");
    uint64_t need = (uint64_t)c->n_materials * kTabPerMat * kNodes;
    if (n_doubles < need) return fail(EMS_ERR_INVALID_ARG, "output too small");
    HIP_TRY(hipMemcpyAsync(out, c->ws + c->L.tables64, 8 * need, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return EMS_OK;
}

ems_status ems_push_primaries(ems_ctx* c, const ems_primary* p, uint64_t n)
{
    ems_status s = check_ready(c);
    if (s != EMS_OK) return s;
    if (n == 0) return EMS_OK;
    if (!p) return fail(EMS_ERR_INVALID_ARG, "null primaries");
    // validate everything before touching any state
    uint64_t new_events = 0;
    std::unordered_map<uint64_t, int> seen;
    for (uint64_t i = 0; i < n; ++i) {
        const ems_primary& q = p[i];
        if (q.type < 0 || q.type > 2) return fail(EMS_ERR_INVALID_ARG, "primary type");
        if (q.slab < 0 || (uint32_t)q.slab >= c->n_slabs) return fail(EMS_ERR_INVALID_ARG, "primary slab");
        if (!(q.T >= c->ecut) || !std::isfinite(q.T)) return fail(EMS_ERR_INVALID_ARG, "primary energy below the cut");
        double un = q.u[0] * q.u[0] + q.u[1] * q.u[1] + q.u[2] * q.u[2];
        if (!(std::fabs(un - 1.0) < 1e-6)) return fail(EMS_ERR_INVALID_ARG, "primary direction not unit");
        if (!(q.r[2] >= c->zp_host[q.slab] && q.r[2] <= c->zp_host[q.slab + 1]) ||
            !(std::fabs(q.r[0]) <= c->half_width && std::fabs(q.r[1]) <= c->half_width))
            return fail(EMS_ERR_INVALID_ARG, "primary position outside its slab");
        if (c->row_of.find(q.event) == c->row_of.end() && seen.emplace(q.event, 1).second) ++new_events;
    }
    if (new_events > c->free_rows.size()) return fail(EMS_ERR_CAPACITY, "not enough free event rows");
    // ring capacity against the last known device consumption (conservative)
    uint64_t consumed = c->last.prim_next;
    if (c->prim_end + n - consumed > c->opt.n_primaries) {
        Snapshot sn;
        s = snapshot_now(c, &sn);
        if (s != EMS_OK) return s;
        consumed = sn.prim_next;
        if (c->prim_end + n - consumed > c->opt.n_primaries) return fail(EMS_ERR_CAPACITY, "primary buffer full");
    }
    Initializer* dst = (Initializer*)(c->ws + c->L.prims);
    uint64_t done = 0;
    while (done < n) {
        if (c->staging_busy) {
            HIP_TRY(hipEventSynchronize(c->staging_ev));
            c->staging_busy = false;
        }
        uint64_t chunk = std::min<uint64_t>(n - done, c->staging_cap);
        for (uint64_t i = 0; i < chunk; ++i) {
            const ems_primary& q = p[done + i];
            uint32_t row;
            s = assign_row(c, q.event, &row);
            if (s != EMS_OK) return s;
            c->row_pending[row] += 1;
            Initializer& r = c->staging[i];
            r.T = q.T;
            r.r[0] = q.r[0]; r.r[1] = q.r[1]; r.r[2] = q.r[2];
            r.u[0] = q.u[0]; r.u[1] = q.u[1]; r.u[2] = q.u[2];
            r.key = q.key;
            r.row = row;
            r.slab = (uint16_t)q.slab;
            r.type = (uint8_t)q.type;
            r.pad = 0;
        }
        // rows first: clearing a row zeroes its live count, which the
        // primaries below then raise
        s = flush_rows(c);
        if (s != EMS_OK) return s;
        // copy into the ring [prim_end, prim_end + chunk) modulo capacity
        uint64_t cap = c->opt.n_primaries;
        uint64_t at = c->prim_end % cap;
        uint64_t first = std::min<uint64_t>(chunk, cap - at);
        HIP_TRY(hipMemcpyAsync(dst + at, c->staging, sizeof(Initializer) * first, hipMemcpyHostToDevice, c->stream));
        if (first < chunk)
            HIP_TRY(hipMemcpyAsync(dst, c->staging + first, sizeof(Initializer) * (chunk - first),
                                   hipMemcpyHostToDevice, c->stream));
        HIP_TRY(hipEventRecord(c->staging_ev, c->stream));
        c->staging_busy = true;
        hipLaunchKernelGGL(k_count_primaries, dim3((chunk + 255) / 256), dim3(256), 0, c->stream, (const Initializer*)dst,
                           cap, c->prim_end, chunk, (unsigned int*)(c->ws + c->L.live), c->L.n_rep - 1,
                           c->L.live_rs);
        HIP_TRY(hipGetLastError());
        c->prim_end += chunk;
        done += chunk;
    }
    hipLaunchKernelGGL(k_set_prim_end, dim3(1), dim3(1), 0, c->stream, (Counters*)(c->ws + c->L.ctr),
                       (unsigned long long)c->prim_end);
    HIP_TRY(hipGetLastError());
    return EMS_OK;
}

ems_status ems_step(ems_ctx* c, uint32_t iterations, ems_counters* out)
{
    ems_status s = check_ready(c);
    if (s != EMS_OK) return s;
    const uint32_t gi = c->opt.graph_iterations > 0 ? (uint32_t)c->opt.graph_iterations : 0;
    uint32_t done = 0;
    while (gi > 0 && iterations - done >= gi) {
        s = launch_batch(c, (int)gi, false);
        if (s != EMS_OK) return s;
        done += gi;
    }
    for (; done < iterations; ++done) {
        s = launch_batch(c, 1, false);
        if (s != EMS_OK) return s;
    }
    if (out) {
        Snapshot sn;
        s = snapshot_now(c, &sn);
        if (s != EMS_OK) return s;
        to_counters(sn, out);
        if (sn.overflow) return fail(EMS_ERR_CAPACITY, "initializer buffer overflow: increase n_initializers");
    }
    return EMS_OK;
}

ems_status ems_run(ems_ctx* c, uint64_t max_iterations, ems_counters* out)
{
    ems_status s = check_ready(c);
    if (s != EMS_OK) return s;
    const int batch = c->opt.graph_iterations > 0 ? c->opt.graph_iterations : 16;
    uint64_t launched = 0;
    uint64_t seq = 0;
    // batches in flight: after launching batch g we wait for the snapshot of batch g-1
    Snapshot done{};
    bool have_done = false;
    bool finished = false;
    int in_flight = 0;
    // tracks alive, queued or pending in the latest snapshot and in the one
    // before it
    uint64_t left = UINT64_MAX, left_before = UINT64_MAX;
    bool draining = false;
    while (!finished) {
        if (launched < max_iterations) {
            // the rest of the work is drained, one drain iteration at a time,
            // once the latest snapshot shows fewer tracks than the threshold
            // and no more than the snapshot before it (the tail of the run,
            // not the ramp of one that starts with few tracks), until a
            // snapshot shows the threshold reached again; the largest
            // threshold drains every iteration from the first
            const bool below = c->drain_threshold > 0 && left < c->drain_threshold;
            draining = c->drain_threshold == UINT32_MAX || (below && (draining || left <= left_before));
            if (draining) {
                // two threads per track left (half of a block's threads own
                // vacant slots); before the first snapshot, all of them
                const uint64_t cap = c->L.drain_threads;
                const uint64_t want = left >= cap ? cap : align_up(std::max<uint64_t>(2 * left, 256), 256);
                launch_drain_any(c, (uint32_t)std::min<uint64_t>(want, cap));
                launch_completions(c);
                HIP_TRY(hipGetLastError());
                launched += 1;
            } else {
                s = launch_batch(c, batch, false);
                if (s != EMS_OK) return s;
                launched += batch;
            }
            int slot = (int)(seq % c->snap_slots);
            launch_snapshot(c, &c->snap[slot]);
            HIP_TRY(hipEventRecord(c->snap_ev[slot], c->stream));
            ++seq;
            ++in_flight;
        }
        if (in_flight >= 2 || launched >= max_iterations) {
            int slot = (int)((seq - in_flight) % c->snap_slots);
            HIP_TRY(hipEventSynchronize(c->snap_ev[slot]));
            done = c->snap[slot];
            // the first snapshot has none before it: no drain decision yet
            left_before = have_done ? left : 0;
            left = (uint64_t)done.n_alive + done.queue_size + (done.prim_end - done.prim_next);
            have_done = true;
            --in_flight;
            if (done.overflow) {
                HIP_TRY(hipStreamSynchronize(c->stream));
                c->last = done;
                if (out) to_counters(done, out);
                return fail(EMS_ERR_CAPACITY, "initializer buffer overflow: increase n_initializers");
            }
            if (done.n_alive == 0 && done.queue_size == 0 && done.prim_next == done.prim_end) finished = true;
            else if (launched >= max_iterations && in_flight == 0) break;
        }
    }
    HIP_TRY(hipStreamSynchronize(c->stream));
    Snapshot fin;
    s = snapshot_now(c, &fin);
    if (s != EMS_OK) return s;
    if (out) to_counters(fin, out);
    if (!finished) return fail(EMS_ERR_STATE, "max_iterations reached before the slots emptied");
    return EMS_OK;
}

ems_status ems_read_counters(ems_ctx* c, ems_counters* out)
{
    if (!c || !out) return fail(EMS_ERR_INVALID_ARG, "null");
    Snapshot sn;
    ems_status s = snapshot_now(c, &sn);
    if (s != EMS_OK) return s;
    to_counters(sn, out);
    return EMS_OK;
}

ems_status ems_last_counters(ems_ctx* c, ems_counters* out)
{
    if (!c || !out) return fail(EMS_ERR_INVALID_ARG, "null");
    to_counters(c->last, out);
    return EMS_OK;
}

ems_status ems_poll_completed(ems_ctx* c, uint64_t* events, uint32_t cap, uint32_t* n)
{
    if (!c || !n || (!events && cap)) return fail(EMS_ERR_INVALID_ARG, "null");
    *n = 0;
    Snapshot sn;
    ems_status s = snapshot_now(c, &sn);
    if (s != EMS_OK) return s;
    // secondaries beyond the initializer buffer were dropped: the events
    // completing now may miss energy, so none is reported
    if (sn.overflow) return fail(EMS_ERR_CAPACITY, "initializer buffer overflow: increase n_initializers");
    uint32_t rows_n = c->opt.max_events;
    uint32_t avail = sn.done_count - c->done_read;
    if (avail > rows_n) {
        // older entries were overwritten; they belonged to registrations that were
        // released without polling (at most rows_n registrations are live at once)
        c->done_read = sn.done_count - rows_n;
        avail = rows_n;
    }
    if (avail == 0) return EMS_OK;
    std::vector<uint64_t> ring(rows_n);
    HIP_TRY(hipMemcpyAsync(ring.data(), c->ws + c->L.done_ring, 8ull * rows_n, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    // entries of an earlier registration of a row (released without polling) are skipped
    uint32_t m = 0, k = 0;
    for (; k < avail && m < cap; ++k) {
        uint64_t e = ring[(c->done_read + k) % rows_n];
        uint32_t row = (uint32_t)e, gen = (uint32_t)(e >> 32);
        if (row < rows_n && c->row_gen[row] == gen && c->row_event[row] != UINT64_MAX) events[m++] = c->row_event[row];
    }
    c->done_read += k;
    *n = m;
    return EMS_OK;
}

ems_status ems_read_edep(ems_ctx* c, uint64_t event, double* per_slab, uint32_t n_slabs, ems_ledger* ledger)
{
    if (!c) return fail(EMS_ERR_INVALID_ARG, "null context");
    auto it = c->row_of.find(event);
    if (it == c->row_of.end()) return fail(EMS_ERR_INVALID_ARG, "unknown event");
    uint32_t row = it->second;
    if (per_slab) {
        if (n_slabs < c->n_slabs) return fail(EMS_ERR_INVALID_ARG, "per_slab too small");
        const uint32_t ms = (uint32_t)c->opt.max_slabs;
        hipLaunchKernelGGL(k_edep_sum, dim3((ms + 255) / 256), dim3(256), 0, c->stream, (const double*)(c->ws + c->L.edep),
                           c->L.n_rep_e, c->L.edep_rs, ms, row, 1u, (double*)(c->ws + c->L.edep_out));
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(per_slab, c->ws + c->L.edep_out, 8ull * c->n_slabs, hipMemcpyDeviceToHost, c->stream));
    }
    if (ledger) {
        hipLaunchKernelGGL(k_ledger_sum, dim3(1), dim3(64), 0, c->stream, (const Ledger*)(c->ws + c->L.ledger),
                           c->L.n_rep, c->L.ledger_rs, row, 1u, (Ledger*)(c->ws + c->L.ledger_out));
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(ledger, c->ws + c->L.ledger_out, sizeof(Ledger), hipMemcpyDeviceToHost, c->stream));
    }
    HIP_TRY(hipStreamSynchronize(c->stream));
    return EMS_OK;
}

ems_status ems_read_all_tallies(ems_ctx* c, double* edep, ems_ledger* ledgers, uint64_t* row_event)
{
    if (!c) return fail(EMS_ERR_INVALID_ARG, "null context");
    uint64_t rows = c->opt.max_events;
    if (edep) {
        // rows are stored with stride max_slabs; return them with stride n_slabs
        std::vector<double> tmp(rows * c->opt.max_slabs);
        const uint32_t ms = (uint32_t)c->opt.max_slabs;
        hipLaunchKernelGGL(k_edep_sum, dim3((uint32_t)((rows * ms + 255) / 256)), dim3(256), 0, c->stream,
                           (const double*)(c->ws + c->L.edep), c->L.n_rep_e, c->L.edep_rs, ms, 0u, (uint32_t)rows,
                           (double*)(c->ws + c->L.edep_out));
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(tmp.data(), c->ws + c->L.edep_out, 8ull * rows * c->opt.max_slabs, hipMemcpyDeviceToHost,
                               c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        for (uint64_t r = 0; r < rows; ++r)
            std::memcpy(edep + r * c->n_slabs, tmp.data() + r * c->opt.max_slabs, 8ull * c->n_slabs);
    }
    if (ledgers) {
        hipLaunchKernelGGL(k_ledger_sum, dim3((uint32_t)((rows + 255) / 256)), dim3(256), 0, c->stream,
                           (const Ledger*)(c->ws + c->L.ledger), c->L.n_rep, c->L.ledger_rs, 0u, (uint32_t)rows,
                           (Ledger*)(c->ws + c->L.ledger_out));
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(ledgers, c->ws + c->L.ledger_out, sizeof(Ledger) * rows, hipMemcpyDeviceToHost,
                               c->stream));
    }
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (row_event) std::memcpy(row_event, c->row_event.data(), 8ull * rows);
    return EMS_OK;
}

ems_status ems_release_events(ems_ctx* c, const uint64_t* events, uint64_t n)
{
    if (!c || (!events && n)) return fail(EMS_ERR_INVALID_ARG, "null");
    // validate all first: nothing is released on error
    std::unordered_map<uint64_t, int> seen;
    for (uint64_t i = 0; i < n; ++i) {
        if (c->row_of.find(events[i]) == c->row_of.end()) return fail(EMS_ERR_INVALID_ARG, "unknown event");
        if (!seen.emplace(events[i], 1).second) return fail(EMS_ERR_INVALID_ARG, "event listed twice");
    }
    for (uint64_t i = 0; i < n; ++i) {
        auto it = c->row_of.find(events[i]);
        uint32_t row = it->second;
        c->row_of.erase(it);
        c->row_event[row] = UINT64_MAX;
        c->row_pending[row] = 0;
        c->row_gen[row] += 1;
        c->reg_pending.push_back(RowReg{UINT64_MAX, row, c->row_gen[row]});
        c->free_rows.push_back(row);
    }
    return flush_rows(c);
}

ems_status ems_release_event(ems_ctx* c, uint64_t event) { return ems_release_events(c, &event, 1); }

// ---------------------------------------------------------------- test hooks
ems_status ems_debug_register_event(ems_ctx* c, uint64_t event, uint32_t* row)
{
    if (!c || !row) return fail(EMS_ERR_INVALID_ARG, "null");
    ems_status s = assign_row(c, event, row);
    if (s != EMS_OK) return s;
    return flush_rows(c);
}

ems_status ems_debug_inject(ems_ctx* c, const ems_track* t, uint64_t n)
{
    ems_status s = check_ready(c);
    if (s != EMS_OK) return s;
    if (n > c->opt.n_slots) return fail(EMS_ERR_CAPACITY, "more tracks than slots");
    for (uint64_t i = 0; i < n; ++i) {
        if (t[i].type < 0) continue;
        if (t[i].type > 2 || t[i].slab < 0 || (uint32_t)t[i].slab >= c->n_slabs || t[i].row >= c->opt.max_events ||
            c->row_event[t[i].row] == UINT64_MAX || !(t[i].T >= c->ecut))
            return fail(EMS_ERR_INVALID_ARG, "invalid injected track");
    }
    ems_track* dt = nullptr;
    HIP_TRY(hipMalloc(&dt, sizeof(ems_track) * (n ? n : 1)));
    if (n) HIP_TRY(hipMemcpyAsync(dt, t, sizeof(ems_track) * n, hipMemcpyHostToDevice, c->stream));
    uint64_t ns = c->opt.n_slots;
    hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(1), 0, c->stream, (Counters*)(c->ws + c->L.ctr));
    if (c->opt.precision == EMS_MIXED)
        hipLaunchKernelGGL(k_inject<float>, dim3((ns + 255) / 256), dim3(256), 0, c->stream, make_dev<float>(c), dt, n);
    else
        hipLaunchKernelGGL(k_inject<double>, dim3((ns + 255) / 256), dim3(256), 0, c->stream, make_dev<double>(c), dt, n);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipFree(dt));
    return EMS_OK;
}

ems_status ems_debug_iterate(ems_ctx* c, uint32_t iterations, int32_t no_init)
{
    ems_status s = check_ready(c);
    if (s != EMS_OK) return s;
    for (uint32_t i = 0; i < iterations; ++i) launch_iteration_any(c, no_init != 0, c->prof_mask != 0);
    launch_completions(c);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(c->stream));
    return EMS_OK;
}

ems_status ems_debug_read_tracks(ems_ctx* c, ems_track* t, uint64_t n)
{
    if (!c || !t) return fail(EMS_ERR_INVALID_ARG, "null");
    if (n > c->opt.n_slots) return fail(EMS_ERR_INVALID_ARG, "n > n_slots");
    if (n == 0) return EMS_OK;
    ems_track* dt = nullptr;
    HIP_TRY(hipMalloc(&dt, sizeof(ems_track) * n));
    if (c->opt.precision == EMS_MIXED)
        hipLaunchKernelGGL(k_read_tracks<float>, dim3((n + 255) / 256), dim3(256), 0, c->stream, make_dev<float>(c), dt, n);
    else
        hipLaunchKernelGGL(k_read_tracks<double>, dim3((n + 255) / 256), dim3(256), 0, c->stream, make_dev<double>(c), dt, n);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(t, dt, sizeof(ems_track) * n, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipFree(dt));
    return EMS_OK;
}

ems_status ems_debug_read_secondaries(ems_ctx* c, ems_track* out, uint64_t cap, uint64_t* n)
{
    if (!c || !n) return fail(EMS_ERR_INVALID_ARG, "null");
    Snapshot sn;
    ems_status s = snapshot_now(c, &sn);
    if (s != EMS_OK) return s;
    uint64_t q = sn.queue_size < c->opt.n_initializers ? sn.queue_size : c->opt.n_initializers;
    *n = q;
    uint64_t m = q < cap ? q : cap;
    if (m == 0 || !out) return EMS_OK;
    ems_track* dt = nullptr;
    HIP_TRY(hipMalloc(&dt, sizeof(ems_track) * m));
    hipLaunchKernelGGL(k_read_queue, dim3((m + 255) / 256), dim3(256), 0, c->stream,
                       (const Initializer*)(c->ws + c->L.queue), m, dt);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(out, dt, sizeof(ems_track) * m, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipFree(dt));
    return EMS_OK;
}

ems_status ems_debug_sort(ems_ctx* c, const uint8_t* keys, uint64_t n, int32_t policy, uint32_t* perm)
{
    if (!c || (!keys && n) || (!perm && n)) return fail(EMS_ERR_INVALID_ARG, "null");
    if (policy != EMS_SORT_PARTITION && policy != EMS_SORT_RADIX) return fail(EMS_ERR_INVALID_ARG, "policy");
    if (n == 0) return EMS_OK;
    if (n > 0xFFFFFFFFull) return fail(EMS_ERR_INVALID_ARG, "n too large");
    const int nb = policy == EMS_SORT_PARTITION ? 16 : 128;
    for (uint64_t i = 0; i < n; ++i)
        if (keys[i] >= nb) return fail(EMS_ERR_INVALID_ARG, "key out of range for the policy");
    uint32_t nt = (uint32_t)((n + kSortTile - 1) / kSortTile);
    uint8_t* dk = nullptr;
    uint32_t *dp = nullptr, *cnt = nullptr, *tot = nullptr;
    auto release = [&]() {
        (void)hipFree(dk);
        (void)hipFree(dp);
        (void)hipFree(cnt);
        (void)hipFree(tot);
    };
    auto try_ = [&](hipError_t e) {
        if (e != hipSuccess) release();
        return e;
    };
    HIP_TRY(try_(hipMalloc(&dk, n)));
    HIP_TRY(try_(hipMalloc(&dp, 4 * n)));
    HIP_TRY(try_(hipMalloc(&cnt, 4ull * 128 * nt)));
    HIP_TRY(try_(hipMalloc(&tot, 4ull * 128)));
    HIP_TRY(try_(hipMemcpyAsync(dk, keys, n, hipMemcpyHostToDevice, c->stream)));
    Dev<double> d{};
    // the same kernels as a sort point of the step loop
    if (nb == 16) {
        hipLaunchKernelGGL((k_sort_hist<double, 16>), dim3(nt), dim3(kSortThreads), 0, c->stream, d, 0, dk, (uint32_t)n,
                           cnt, nt);
        hipLaunchKernelGGL((k_sort_scan<16>), dim3(16), dim3(256), 0, c->stream, cnt, nt, (const Counters*)nullptr, tot,
                           0u);
        hipLaunchKernelGGL((k_sort_scatter<double, 16>), dim3(nt), dim3(kSortThreads), 0, c->stream, d, 0, dk,
                           (uint32_t)n, cnt, nt, (const uint32_t*)tot, dp);
    } else {
        hipLaunchKernelGGL((k_sort_hist<double, 128>), dim3(nt), dim3(kSortThreads), 0, c->stream, d, 1, dk,
                           (uint32_t)n, cnt, nt);
        hipLaunchKernelGGL((k_sort_scan<128>), dim3(128), dim3(256), 0, c->stream, cnt, nt, (const Counters*)nullptr,
                           tot, 0u);
        hipLaunchKernelGGL((k_sort_scatter<double, 128>), dim3(nt), dim3(kSortThreads), 0, c->stream, d, 1, dk,
                           (uint32_t)n, cnt, nt, (const uint32_t*)tot, dp);
    }
    HIP_TRY(try_(hipGetLastError()));
    HIP_TRY(try_(hipMemcpyAsync(perm, dp, 4 * n, hipMemcpyDeviceToHost, c->stream)));
    HIP_TRY(try_(hipStreamSynchronize(c->stream)));
    release();
    return EMS_OK;
}

ems_status ems_sort_keys_noalloc(ems_ctx* c, const uint8_t* keys, uint64_t n, int32_t policy, uint32_t* perm)
{
    if (!c) return fail(EMS_ERR_INVALID_ARG, "null context");
    if (policy != EMS_SORT_PARTITION && policy != EMS_SORT_RADIX) return fail(EMS_ERR_INVALID_ARG, "policy");
    if (n == 0) return EMS_OK;
    if (!keys || !perm) return fail(EMS_ERR_INVALID_ARG, "null keys or perm");
    if (n > kNoAllocMaxKeys)
        return fail(EMS_ERR_CAPACITY, "ems_sort_keys_noalloc sorts at most 2^23 keys (fixed scratch of 4 MiB)");
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != c->device) return fail(EMS_ERR_STATE, "the context's device must be current");
    uint32_t* ptr = scratch_on_device(dev);
    if (!ptr) return EMS_ERR_DEVICE;
    const uint32_t nt = (uint32_t)((n + kSortTile - 1) / kSortTile);
    // counts [bin][tile] and the bin totals after them; every word the sort
    // reads is written by this call's histogram and scan kernels first, so
    // nothing needs clearing between calls
    uint32_t* cnt = ptr;
    uint32_t* tot = ptr + 128 * kNoAllocTiles;
    Dev<double> d{};
    if (policy == EMS_SORT_PARTITION) {
        hipLaunchKernelGGL((k_sort_hist<double, 16>), dim3(nt), dim3(kSortThreads), 0, c->stream, d, 0, keys,
                           (uint32_t)n, cnt, nt);
        hipLaunchKernelGGL((k_sort_scan<16>), dim3(16), dim3(256), 0, c->stream, cnt, nt, (const Counters*)nullptr,
                           tot, 0u);
        hipLaunchKernelGGL((k_sort_scatter<double, 16>), dim3(nt), dim3(kSortThreads), 0, c->stream, d, 0, keys,
                           (uint32_t)n, (const uint32_t*)cnt, nt, (const uint32_t*)tot, perm);
    } else {
        hipLaunchKernelGGL((k_sort_hist<double, 128>), dim3(nt), dim3(kSortThreads), 0, c->stream, d, 1, keys,
                           (uint32_t)n, cnt, nt);
        hipLaunchKernelGGL((k_sort_scan<128>), dim3(128), dim3(256), 0, c->stream, cnt, nt, (const Counters*)nullptr,
                           tot, 0u);
        hipLaunchKernelGGL((k_sort_scatter<double, 128>), dim3(nt), dim3(kSortThreads), 0, c->stream, d, 1, keys,
                           (uint32_t)n, (const uint32_t*)cnt, nt, (const uint32_t*)tot, perm);
    }
    HIP_TRY(hipGetLastError());
    return EMS_OK;
}

ems_status ems_set_tuning(ems_ctx* c, const ems_tuning* t)
{
    if (!c || !t) return fail(EMS_ERR_INVALID_ARG, "null");
    if (t->sort_policy < 0 || t->sort_policy > 3) return fail(EMS_ERR_INVALID_ARG, "sort_policy");
    for (int i = 0; i < 16; ++i) {
        int b = t->block[i];
        if (b != 0 && (b < 64 || b > 512 || (b % 64) != 0))
            return fail(EMS_ERR_INVALID_ARG, "block sizes must be 0 or a multiple of 64 in [64, 512]");
    }
    if (t->drain_threshold > 0 && t->drain_steps == 0) return fail(EMS_ERR_INVALID_ARG, "drain_steps must be > 0");
    if (c->opt.deterministic && (t->sort_policy == EMS_SORT_QUEUE || t->drain_threshold > 0))
        return fail(EMS_ERR_INVALID_ARG, "deterministic appends do not combine with the queue policy or the drain");
    c->policy = t->sort_policy;
    c->tail_threshold = t->tail_threshold;
    c->phase_sort[0] = t->phase_sort[0];
    c->phase_sort[1] = t->phase_sort[1];
    c->drain_threshold = t->drain_threshold;
    c->drain_steps = t->drain_steps;
    c->reuse_parent = t->reuse_parent_slot ? 1u : 0u;
    c->fuse_interactions = t->fuse_interactions ? 1u : 0u;
    c->fuse_along = t->fuse_along ? 1u : 0u;
    for (int i = 0; i < 16; ++i) c->block[i] = t->block[i];
    return drop_graph(c);
}

ems_status ems_get_tuning(ems_ctx* c, ems_tuning* t)
{
    if (!c || !t) return fail(EMS_ERR_INVALID_ARG, "null");
    t->sort_policy = c->policy;
    t->tail_threshold = c->tail_threshold;
    t->drain_threshold = c->drain_threshold;
    t->drain_steps = c->drain_steps;
    t->reuse_parent_slot = c->reuse_parent;
    t->fuse_interactions = c->fuse_interactions;
    t->fuse_along = c->fuse_along;
    t->phase_sort[0] = c->phase_sort[0];
    t->phase_sort[1] = c->phase_sort[1];
    for (int i = 0; i < 16; ++i) t->block[i] = c->block[i];
    return EMS_OK;
}

ems_status ems_profile_enable(ems_ctx* c, int32_t enable)
{
    if (!c) return fail(EMS_ERR_INVALID_ARG, "null");
    c->prof_mask = (uint32_t)enable;
    return EMS_OK;
}

ems_status ems_profile_read(ems_ctx* c, const char** names, double* total_ms, uint64_t* launches, uint32_t cap,
                            uint32_t* n)
{
    if (!c || !n) return fail(EMS_ERR_INVALID_ARG, "null");
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (auto& e : c->prof_events) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e.second.first, e.second.second);
        c->prof_ms[e.first] += ms;
        c->prof_n[e.first] += 1;
        (void)hipEventDestroy(e.second.first);
        (void)hipEventDestroy(e.second.second);
    }
    c->prof_events.clear();
    uint32_t m = cap < (uint32_t)R_NUM ? cap : (uint32_t)R_NUM;
    for (uint32_t i = 0; i < m; ++i) {
        if (names) names[i] = kRoleNames[i];
        if (total_ms) total_ms[i] = c->prof_ms[i];
        if (launches) launches[i] = c->prof_n[i];
        c->prof_ms[i] = 0.0;
        c->prof_n[i] = 0;
    }
    *n = m;
    return EMS_OK;
}

}  // extern "C"
