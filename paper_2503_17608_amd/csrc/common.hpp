// Shared host/device definitions of the step-loop library: state layout,
// action codes, counters and small device helpers.
//
// Track state is a struct of arrays over n_slots (paper, "Stepping
// algorithm"): a per-track quantity is its own array so that a kernel
// reading one field over many slots streams it contiguously from HBM.  The
// exception is the group that every step and every interaction reads and
// writes together (position, direction, kinetic energy, random-number key):
// it shares one 64-byte record per slot.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ems {

// ---- physical constants (CODATA 2018) ---------------------------------------
constexpr double kMe = 0.51099895;            // electron rest energy [MeV]
constexpr double kRe = 2.8179403262e-13;      // classical electron radius [cm]
constexpr double kAlpha = 1.0 / 137.035999084;
constexpr double kNA = 6.02214076e23;         // [1/mol]
constexpr double kCk = 2.99792458;            // p[MeV] = kCk * B[T] * radius[cm]
constexpr double kPlasma = 28.816;            // hbar omega_p = 28.816 sqrt(rho Z / A) eV
constexpr double kPi = 3.14159265358979323846;

// ---- transport parameters -----------------------------------------------------
constexpr int kNodes = 181;                   // table nodes: 1 keV .. 1 TeV, 20 per decade
constexpr int kTabPerMat = 8;
constexpr double kEmin = 1.0e-3;
constexpr double kRhoRange = 0.2;             // step <= rho * range ...
constexpr double kRFinal = 0.01;              // ... but not below r_f [cm]
constexpr double kDChord = 0.0025;            // field substep sagitta [cm]
constexpr double kDInt = 1.0e-5;              // boundary-search tolerance [cm]
constexpr int kMaxSearch = 10;
constexpr int kMaxTrials = 1000;
constexpr uint32_t kMaxSteps = 1000000u;

// table indices within a material
enum : int { TB_COMPTON = 0, TB_PHOTO, TB_PAIR, TB_MOLLER, TB_BHABHA, TB_BREMS, TB_RANGE_EM, TB_RANGE_EP };
// particle types stored in the state; kDead marks a vacant slot
enum : uint8_t { kGamma = 0, kElectron = 1, kPositron = 2, kDead = 3 };
// discrete actions: the six sampled processes, then annihilation at rest (a
// positron that stopped in its along-step; it is not chosen by cross section)
enum : int { P_COMPTON = 0, P_PHOTO, P_PAIR, P_MOLLER, P_BHABHA, P_BREMS, P_ANNIH, kNumProc };

// Next-action codes (the sort key).  The along-step action follows from the
// particle type and the field; interaction actions are set by the along-step
// kernels.
enum : uint8_t {
    A_IDLE = 0,        // alive, no work this phase
    A_NEUTRAL = 1,     // straight-line along-step of a photon
    A_CHARGED = 2,     // straight-line along-step with continuous loss (no field)
    A_FIELD = 3,       // field propagation (also a paused step)
    A_PROC0 = 4,       // + process index: discrete interaction
    A_ANNIH = A_PROC0 + P_ANNIH,
    A_NUM = A_PROC0 + kNumProc,
    A_NONE = 0xFF      // vacant slot
};

// flags byte
enum : uint8_t {
    F_DREW = 1,        // the interaction-length uniform (index 0) was drawn this step
    F_LOSS = 2,        // the physics step limit is the energy-loss limit
    F_PAUSED = 4,      // field step paused at the substep cap
    // the stop of a positron waiting for annihilation at rest was counted as
    // a step already (step-guard stop): the annihilation adds no step
    F_COUNTED = 32,
};


// faces of a slab box
enum : int { F_NONE = 0, F_ZLO, F_ZHI, F_XLO, F_XHI, F_YLO, F_YHI };

// Track initializer: the minimal record to start a track (paper, "Stepping
// algorithm").  80 bytes, written by interaction kernels and read once by the
// initialization kernel; records are contiguous per wave.
struct alignas(16) Initializer {
    double T;
    double r[3];
    double u[3];
    uint64_t key;
    uint32_t row;
    uint16_t slab;
    uint8_t type;
    uint8_t pad;
};
static_assert(sizeof(Initializer) == 80, "initializer layout");

// per-event ledger (same layout as ems_ledger)
struct Ledger {
    double escaped;
    unsigned long long n_pair, n_annih, steps;
    unsigned long long n_sec[3];
    unsigned long long n_guard, n_reject_cap;
};
static_assert(sizeof(Ledger) == 72, "ledger layout");

// device-resident loop counters
struct Counters {
    unsigned long long queue_size;     // secondaries waiting in the initializer buffer
    unsigned long long prim_next;      // next pending primary
    unsigned long long prim_end;       // end of pushed primaries
    unsigned long long iterations;
    unsigned int n_vac;                // vacancies found this iteration
    unsigned int n_alive;              // live tracks at the start of this iteration
    unsigned int overflow;
    unsigned int n_take_q;             // initializers taken from the queue this iteration
    unsigned int n_take_p;             // primaries taken this iteration
    unsigned long long q_base;         // first queue index taken (top - n_take_q)
    unsigned long long p_base;
    unsigned int range_off[16];        // sorted mode: start of each action's index range
    unsigned int range_cnt[16];
    unsigned int list_cnt[16];         // queue policy: entries of each interaction list
    unsigned int alive_before;         // live tracks found by the vacancy pass (before the fill)
    unsigned int done_count;           // events completed so far (entries written to the ring)
    unsigned int phase_sorted;         // reordering this iteration: bit 0 sort point 1, bit 1 sort point 2
    unsigned long long sec_base;       // deterministic appends: buffer size before this iteration's appends
    unsigned int n_take_lo;            // taken initializers that went to the lowest vacancies (the rest to
                                       // the highest): the charged ones with the partitioned fill, else all
    unsigned int n_take_hi;            // partitioned fill by block reservations: neutral ones placed so far
};

// work counter indices
enum : int {
    W_REUSE = 0, W_INIT = 1, W_PRE = 2, W_SORT = 3, W_NEUTRAL = 4, W_CHARGED = 5, W_FIELD = 6, W_PROC0 = 7,
    W_PAUSED = W_PROC0 + kNumProc, W_SUBSTEPS, W_DRAIN
};
// partial-counter slots: [0, kNumWork) work per kernel, [kStepsSlot, kNumW)
// completed steps of the tracks each kernel retired (one slot per kernel,
// since kernels of an iteration may run concurrently: such a slot has a
// single writer; the pre-step and slot-reuse roles, which concurrent
// kernels share, are updated atomically)
constexpr int kNumWork = W_DRAIN + 1;
constexpr int kStepsSlot = kNumWork;
constexpr int kNumW = 2 * kNumWork;
static_assert(W_DRAIN < kNumWork, "work counter slots");
constexpr uint32_t kDrainThreadsMax = 1u << 16;   // drain kernel threads (8 stack records each, per block)
constexpr int kDrainDepth = 8;                     // private secondary stack depth per drain thread
constexpr uint32_t kDrainStepsDefault = 4096;      // steps per drain thread and launch
constexpr int kDrainSubsteps = 1024;               // field substeps per drain trip before a pause
constexpr int kDrainBurst = 4;                     // steps per track and drain round

// Host-visible snapshot copied to pinned memory after each batch
struct Snapshot {
    unsigned long long queue_size, prim_next, prim_end, iterations, steps_done;
    unsigned int n_vac, n_alive, overflow, done_count;
    unsigned long long work[kNumWork];
};

// ---- Philox4x64-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers:
// as easy as 1, 2, 3", SC'11) ----------------------------------------------------
struct U64x4 { uint64_t w[4]; };

// Full 64 x 64 -> 128-bit product from four 32 x 32 -> 64-bit partial
// products (schoolbook), so that the low and high halves share them.
__device__ __forceinline__ void mulhilo64(uint64_t a, uint64_t b, uint64_t& lo, uint64_t& hi)
{
    const uint64_t a0 = (uint32_t)a, a1 = a >> 32, b0 = (uint32_t)b, b1 = b >> 32;
    const uint64_t p00 = a0 * b0;
    const uint64_t p10 = a1 * b0 + (p00 >> 32);          // < 2^64: no carry is lost
    const uint64_t p01 = a0 * b1 + (uint32_t)p10;        // < 2^64
    hi = a1 * b1 + (p10 >> 32) + (p01 >> 32);
    lo = (p01 << 32) | (uint32_t)p00;
}

__device__ __forceinline__ U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                               uint64_t k0, uint64_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t m0 = 0xD2E7470EE14C6C93ULL, m1 = 0xCA5A826395121157ULL;
        uint64_t lo0, hi0, lo1, hi1;
        mulhilo64(m0, c0, lo0, hi0);
        mulhilo64(m1, c2, lo1, hi1);
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B97F4A7C15ULL;
        k1 += 0xBB67AE8584CAA73BULL;
    }
    U64x4 o;
    o.w[0] = c0; o.w[1] = c1; o.w[2] = c2; o.w[3] = c3;
    return o;
}

template <class R> __device__ __forceinline__ R unit_from(uint64_t w);
template <> __device__ __forceinline__ double unit_from<double>(uint64_t w)
{
    return ((double)(w >> 12) + 0.5) * 0x1p-52;
}
template <> __device__ __forceinline__ float unit_from<float>(uint64_t w)
{
    return ((float)(uint32_t)(w >> 41) + 0.5f) * 0x1p-23f;
}

// Uniforms of one track step: uniform j is word j&3 of the Philox block
// (key, step, j>>2, domain 0) under key (seed, event).
template <class R>
struct StepRng {
    uint64_t k0, k1, key, step;
    int j;
    int have;          // block index cached in b0..b3, -1 none
    uint64_t b0, b1, b2, b3;
    __device__ StepRng(uint64_t seed, uint64_t event, uint64_t track_key, uint64_t step_, int j0)
        : k0(seed), k1(event), key(track_key), step(step_), j(j0), have(-1), b0(0), b1(0), b2(0), b3(0) {}
    __device__ __forceinline__ R next()
    {
        int b = j >> 2;
        if (b != have) {
            U64x4 o = philox4x64_10(key, step, (uint64_t)b, 0, k0, k1);
            b0 = o.w[0]; b1 = o.w[1]; b2 = o.w[2]; b3 = o.w[3];
            have = b;
        }
        int q = j & 3;
        uint64_t w = q == 0 ? b0 : (q == 1 ? b1 : (q == 2 ? b2 : b3));
        ++j;
        return unit_from<R>(w);
    }
};

__device__ __forceinline__ uint64_t child_key(uint64_t seed, uint64_t event, uint64_t key, uint64_t step, int ordinal)
{
    return philox4x64_10(key, step, (uint64_t)ordinal, 1, seed, event).w[0];
}

// ---- math wrappers per precision ------------------------------------------------
__device__ __forceinline__ double m_log(double x) { return log(x); }
__device__ __forceinline__ float m_log(float x) { return logf(x); }
__device__ __forceinline__ double m_exp(double x) { return exp(x); }
__device__ __forceinline__ float m_exp(float x) { return expf(x); }
__device__ __forceinline__ double m_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float m_sqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double m_floor(double x) { return floor(x); }
__device__ __forceinline__ float m_floor(float x) { return floorf(x); }
__device__ __forceinline__ void m_sincos(double x, double* s, double* c) { sincos(x, s, c); }
__device__ __forceinline__ void m_sincos(float x, float* s, float* c) { sincosf(x, s, c); }
__device__ __forceinline__ double m_max(double a, double b) { return fmax(a, b); }
__device__ __forceinline__ float m_max(float a, float b) { return fmaxf(a, b); }
__device__ __forceinline__ double m_min(double a, double b) { return fmin(a, b); }
__device__ __forceinline__ float m_min(float a, float b) { return fminf(a, b); }

}  // namespace ems
