/*
 * Oracle: plain, slow, history-based CPU transporter of electromagnetic showers.
 * TEST INFRASTRUCTURE ONLY -- only tests/, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library.  It shares no code with the
 * device library.
 *
 * What it computes.  The paper (arXiv 2503.17608, "Stepping algorithm") moves
 * from history-based transport -- one particle followed from birth to death,
 * secondaries stacked -- to a step-based loop over actions on a track array.
 * Both do the same per-track work in a different order.  With random numbers
 * keyed by (event, track key, step) rather than by track slot, every track's
 * history is a pure function of its initial state, so the step-based result is
 * exactly the history-based one up to floating-point rounding.  This file is
 * the history-based definition: one event at a time, a LIFO stack of
 * secondaries, every step taken by the rules below.
 *
 * Step rules (per track, step index k, draw index j starting at 0):
 *  S1  n_lambda unset -> n_lambda = -ln U_j.
 *  S2  Sigma(T) = sum of per-process macroscopic cross sections (tables).
 *      s_int = n_lambda / Sigma.
 *  S3  charged: R = R(T); s_loss = R if R <= r_f else max(r_f, rho R);
 *      s_phys = min(s_int, s_loss) (loss-limited only if s_loss < s_int).
 *  S4  geometry: straight line to the slab's exit plane / lateral wall, or the
 *      uniform-field Runge-Kutta propagation (field steps are split into
 *      substeps -- "Reducing load imbalance"; the paper caps substeps per step
 *      iteration and resumes the step later, which does not change the
 *      history, so this oracle runs every step to completion).
 *      s_geo <= s_phys -> geometry-limited (ties go to geometry).
 *  S5  move; snap to the crossed plane.
 *  S6  charged: T' = R^-1(R(T) - s); deposit T - T'.  Range exhausted or
 *      T' < Ec: deposit all of T and stop (positron: annihilate at rest).
 *  S7  n_lambda -= s * Sigma(T_pre).
 *  S7b optional multiple scattering: a charged track that is still in the
 *      stack after S6 is deflected (see msc_deflect).
 *  S8  boundary: slab +- 1 or escape.  Interaction: U_j * Sigma(T') against
 *      cumulative sigma_i(T'); sample; n_lambda unset.
 *  S9  particles below Ec after an interaction deposit locally; secondaries
 *      below Ec are never created (positrons annihilate at the vertex).
 *  S10 k += 1; k > 10^6 -> stop (guard).
 *
 * Random numbers: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11), key =
 * (seed, event), counter = (track key, step, block, domain).  Uniform j of a
 * step is word j&3 of block j>>2 of domain 0, mapped to ((w>>12)+0.5)*2^-52.
 * Child keys: word 0 of domain 1 at counter (parent key, parent step,
 * ordinal).  Annihilation at rest: domain 4, block 0.  Multiple
 * scattering: domain 5, block 0.
 *
 * Units: MeV, cm, tesla.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_ME 0.51099895            /* electron rest energy [MeV] */
#define ORC_CK 2.99792458            /* p[MeV] = ORC_CK * B[T] * radius[cm] */
#define ORC_NNODES 181
#define ORC_NTAB 8
#define ORC_RHO_RANGE 0.2
#define ORC_R_FINAL 0.01             /* cm */
#define ORC_DCHORD 0.0025            /* cm, chord sagitta for the field substep */
#define ORC_DINT 1.0e-5              /* cm, boundary-search tolerance */
#define ORC_MAX_SEARCH 10
#define ORC_MAX_TRIALS 1000
#define ORC_MAX_STEPS 1000000u
#define ORC_PI 3.14159265358979323846

enum { GAMMA = 0, ELECTRON = 1, POSITRON = 2 };
enum { P_COMPTON = 0, P_PHOTO = 1, P_PAIR = 2, P_MOLLER = 3, P_BHABHA = 4, P_BREMS = 5 };
enum { T_COMPTON = 0, T_PHOTO, T_PAIR, T_MOLLER, T_BHABHA, T_BREMS, T_RANGE_EM, T_RANGE_EP };
enum { OUT_INTERACT = 0, OUT_LOSS = 1, OUT_BOUNDARY = 2, OUT_ESCAPE = 3, OUT_STOP = 4, OUT_GUARD = 5,
       OUT_NO_INTERACT = 6 };
enum { F_NONE = 0, F_ZLO, F_ZHI, F_XLO, F_XHI, F_YLO, F_YHI };

typedef struct {
    int32_t n_slabs;
    int32_t n_materials;
    const double* z_planes;        /* n_slabs + 1, increasing */
    const int32_t* slab_material;  /* n_slabs */
    double half_width;             /* |x|, |y| <= half_width */
    double B[3];                   /* uniform field [T] */
    const double* tables;          /* [n_materials][8][181] */
    double ecut;                   /* production = tracking cut [MeV] */
    uint64_t seed;
    int32_t no_discrete;           /* test hook: 1 = no discrete processes (CSDA) */
    int32_t msc;                   /* 1 = multiple-scattering deflection (S7b) */
    const double* x0_cm;           /* radiation length of each material [cm] */
} orc_problem;

typedef struct {
    uint64_t event;
    uint64_t key;
    int32_t type;
    int32_t slab;
    uint32_t step;
    int32_t alive;
    double T;
    double nl;                     /* remaining mean free paths; < 0 = unset */
    double r[3];
    double u[3];
} orc_track;

#define ORC_MAX_SEC 4
typedef struct {
    int32_t outcome;
    int32_t process;
    int32_t face;
    int32_t dep_slab;
    double step_len;
    double edep;
    double escaped;
    int32_t n_pair;
    int32_t n_annih;
    int32_t n_sec;
    int32_t reject_capped;
    int32_t drew_u0;
    int32_t n_draws;
    orc_track sec[ORC_MAX_SEC];
} orc_step_result;

typedef struct {
    double escaped;
    uint64_t n_pair, n_annih, steps;
    uint64_t n_sec[3];
    uint64_t n_guard, n_reject_cap;
} orc_ledger;

/* ------------------------------------------------------------------ decision margins
 * Flip diagnosis (test infrastructure).  Every comparison that steers the
 * control flow of a step notes how close its two sides were, |a - b| / scale,
 * with a scale that matches how each side's rounding error grows (the larger
 * operand; 1 for uniforms and direction components; max(|plane|, 1 cm) for
 * positions against planes).  The smallest margin of a step and its kind say
 * how far the step was from taking another discrete decision.  Recording is
 * off (a null pointer) except in orc_step_margin and orc_trace_event; it reads
 * values only and changes nothing that the step computes. */
enum {
    M_NONE = 0, M_CUT_START, M_THRESHOLD, M_LOSS_VS_INT, M_RANGE_FINAL, M_GEO_VS_PHYS, M_FACE_TIE, M_DIR_SIGN,
    M_CHORD_BEYOND, M_CHORD_FACE_TIE, M_CHORD_AT_START, M_NEAR_FACE, M_SEARCH_ACCEPT, M_LAST_SUBSTEP,
    M_CUT_AFTER_LOSS, M_PROCESS, M_REJECT, M_BRANCH, M_SECONDARY_CUT, M_ROTATE_POLE
};
typedef struct {
    double margin;
    int32_t kind;
    int32_t n_notes;
} orc_margin;

static __thread orc_margin* g_margin = NULL;

static void note(int kind, double a, double b, double scale)
{
    if (!g_margin) return;
    g_margin->n_notes += 1;
    double m = scale > 0.0 ? fabs(a - b) / scale : INFINITY;
    if (m < g_margin->margin) {
        g_margin->margin = m;
        g_margin->kind = kind;
    }
}

/* relative to the larger operand */
static void note_rel(int kind, double a, double b)
{
    note(kind, a, b, fmax(fabs(a), fabs(b)));
}

/* a sign test of a value that is exactly zero only by construction (a
 * direction component that the field never changes, a chord starting on the
 * plane it was snapped to): an exact zero is the same on any machine */
static void note_sign(int kind, double a, double scale)
{
    if (a != 0.0) note(kind, a, 0.0, scale);
}

/* ------------------------------------------------------------------ Philox */
static void mulhilo64(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo)
{
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

/* Philox4x64 with 10 rounds: each round multiplies counter words 0 and 2 by
 * the two round multipliers, mixes the high halves with the other words and
 * the key, and bumps the key by the two Weyl constants between rounds. */
void orc_philox4x64(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4])
{
    uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(0xD2E7470EE14C6C93ULL, c0, &hi0, &lo0);
        mulhilo64(0xCA5A826395121157ULL, c2, &hi1, &lo1);
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        uint64_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B97F4A7C15ULL;
        k1 += 0xBB67AE8584CAA73BULL;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static double to_unit(uint64_t w) { return ((double)(w >> 12) + 0.5) * 0x1p-52; }

static uint64_t philox_word(const orc_problem* pb, uint64_t event, uint64_t a, uint64_t b,
                            uint64_t c, uint64_t domain, int word)
{
    uint64_t ctr[4] = {a, b, c, domain}, key[2] = {pb->seed, event}, out[4];
    orc_philox4x64(ctr, key, out);
    return out[word];
}

/* uniform number j of the current step of track t */
static double draw(const orc_problem* pb, const orc_track* t, int* j)
{
    int jj = (*j)++;
    return to_unit(philox_word(pb, t->event, t->key, t->step, (uint64_t)(jj >> 2), 0, jj & 3));
}

static uint64_t child_key(const orc_problem* pb, uint64_t event, uint64_t key, uint32_t step, int ordinal)
{
    return philox_word(pb, event, key, step, (uint64_t)ordinal, 1, 0);
}

/* ------------------------------------------------------------------ tables */
static double log_e0(void) { return log(1.0e-3); }
static double dlog(void) { return log(10.0) / 20.0; }

static const double* tab(const orc_problem* pb, int mat, int which)
{
    return pb->tables + ((size_t)mat * ORC_NTAB + (size_t)which) * ORC_NNODES;
}

/* linear interpolation in ln T */
static double lookup(const double* v, double T)
{
    double t = (log(T) - log_e0()) / dlog();
    double fl = floor(t);
    int i = (int)fl;
    if (fl < 0.0) i = 0;
    if (fl > ORC_NNODES - 2) i = ORC_NNODES - 2;
    return v[i] + (t - (double)i) * (v[i + 1] - v[i]);
}

/* exact inverse of the piecewise-linear range map: upper_bound then linear in ln T */
static double inverse_range(const double* R, double r)
{
    int lo = 0, hi = ORC_NNODES;          /* first index with R[idx] > r */
    while (lo < hi) {
        int mid = (lo + hi) / 2;
        if (R[mid] > r) hi = mid; else lo = mid + 1;
    }
    int i = lo - 1;
    if (i < 0) i = 0;
    if (i > ORC_NNODES - 2) i = ORC_NNODES - 2;
    double t = (double)i + (r - R[i]) / (R[i + 1] - R[i]);
    return exp(log_e0() + t * dlog());
}

static int n_procs(int type) { return type == GAMMA ? 3 : 2; }

static int proc_of(int type, int n)
{
    static const int procs[3][3] = {{P_COMPTON, P_PHOTO, P_PAIR}, {P_MOLLER, P_BREMS, -1}, {P_BHABHA, P_BREMS, -1}};
    return procs[type][n];
}

/* per-process macroscopic cross section, zero at and below the process threshold */
static double xs(const orc_problem* pb, int mat, int proc, double T)
{
    switch (proc) {
    case P_COMPTON: return lookup(tab(pb, mat, T_COMPTON), T);
    case P_PHOTO:   return lookup(tab(pb, mat, T_PHOTO), T);
    case P_PAIR:    note_rel(M_THRESHOLD, T, 2.0 * ORC_ME);
                    return T <= 2.0 * ORC_ME ? 0.0 : lookup(tab(pb, mat, T_PAIR), T);
    case P_MOLLER:  note_rel(M_THRESHOLD, T, 2.0 * pb->ecut);
                    return T <= 2.0 * pb->ecut ? 0.0 : lookup(tab(pb, mat, T_MOLLER), T);
    case P_BHABHA:  note_rel(M_THRESHOLD, T, pb->ecut);
                    return T <= pb->ecut ? 0.0 : lookup(tab(pb, mat, T_BHABHA), T);
    case P_BREMS:   note_rel(M_THRESHOLD, T, pb->ecut);
                    return T <= pb->ecut ? 0.0 : lookup(tab(pb, mat, T_BREMS), T);
    }
    return 0.0;
}

static double total_xs(const orc_problem* pb, int mat, int type, double T)
{
    if (pb->no_discrete) return 0.0;
    double s = 0.0;
    for (int n = 0; n < n_procs(type); ++n) s += xs(pb, mat, proc_of(type, n), T);
    return s;
}

static const double* range_tab(const orc_problem* pb, int mat, int type)
{
    return tab(pb, mat, type == POSITRON ? T_RANGE_EP : T_RANGE_EM);
}

/* ------------------------------------------------------------------ vectors */
static void normalize(double v[3])
{
    double n = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    v[0] /= n; v[1] /= n; v[2] /= n;
}

/* rotate direction u by polar cosine c and azimuth phi */
static void rotate(const double u[3], double c, double phi, double out[3])
{
    if (c > 1.0) c = 1.0;
    if (c < -1.0) c = -1.0;
    double s = sqrt(1.0 - c * c);
    double cp = cos(phi), sp = sin(phi);
    double a = sqrt(1.0 - u[2] * u[2]);
    note(M_ROTATE_POLE, a, 1.0e-10, 1.0);
    if (a > 1.0e-10) {
        out[0] = u[0] * c + s * (u[0] * u[2] * cp - u[1] * sp) / a;
        out[1] = u[1] * c + s * (u[1] * u[2] * cp + u[0] * sp) / a;
        out[2] = u[2] * c - a * s * cp;
    } else {
        out[0] = s * cp;
        out[1] = s * sp;
        out[2] = (u[2] >= 0.0 ? 1.0 : -1.0) * c;
    }
}

/* ------------------------------------------------------------------ results */
static void deposit(orc_step_result* res, double e) { res->edep += e; }

static void add_secondary(orc_step_result* res, const orc_track* parent, int type, double T,
                          const double u[3], uint64_t key)
{
    orc_track* s = &res->sec[res->n_sec++];
    memset(s, 0, sizeof(*s));
    s->event = parent->event;
    s->key = key;
    s->type = type;
    s->slab = parent->slab;
    s->step = 0;
    s->alive = 1;
    s->T = T;
    s->nl = -1.0;
    memcpy(s->r, parent->r, sizeof(s->r));
    memcpy(s->u, u, sizeof(s->u));
}

/* Positron annihilation at rest: two photons of m_e c^2 back to back,
 * isotropic; deposited locally when m_e c^2 is below the cut. */
static void annihilate(const orc_problem* pb, const orc_track* pos, uint64_t key, uint32_t step,
                       orc_step_result* res)
{
    res->n_annih += 1;
    if (ORC_ME < pb->ecut) {
        deposit(res, 2.0 * ORC_ME);
        return;
    }
    uint64_t ctr[4] = {key, step, 0, 4}, k[2] = {pb->seed, pos->event}, w[4];
    orc_philox4x64(ctr, k, w);
    double cost = 2.0 * to_unit(w[0]) - 1.0;
    double phi = 2.0 * ORC_PI * to_unit(w[1]);
    double sint = sqrt(1.0 - cost * cost);
    double v[3] = {sint * cos(phi), sint * sin(phi), cost};
    double mv[3] = {-v[0], -v[1], -v[2]};
    add_secondary(res, pos, GAMMA, ORC_ME, v, child_key(pb, pos->event, key, step, 2));
    add_secondary(res, pos, GAMMA, ORC_ME, mv, child_key(pb, pos->event, key, step, 3));
}

/* a charged lepton stops: deposit its kinetic energy; positrons annihilate */
static void stop_track(const orc_problem* pb, orc_track* t, orc_step_result* res)
{
    deposit(res, t->T);
    if (t->type == POSITRON) annihilate(pb, t, t->key, t->step, res);
    t->T = 0.0;
    t->alive = 0;
}

/* ------------------------------------------------------------------ samplers */
static void compton(const orc_problem* pb, orc_track* t, int* j, orc_step_result* res)
{
    double E = t->T, kap = E / ORC_ME;
    double e0 = 1.0 / (1.0 + 2.0 * kap), e0sq = e0 * e0;
    double a1 = -log(e0), a2 = 0.5 * (1.0 - e0sq);
    double eps = 1.0, omc = 0.0;
    for (int trial = 0; trial < ORC_MAX_TRIALS; ++trial) {
        double a = draw(pb, t, j), b = draw(pb, t, j), c = draw(pb, t, j);
        note(M_BRANCH, a * (a1 + a2), a1, a1 + a2);
        if (a * (a1 + a2) < a1) eps = exp(-a1 * b);
        else eps = sqrt(e0sq + (1.0 - e0sq) * b);
        omc = (1.0 - eps) / (kap * eps);
        double sin2 = omc * (2.0 - omc);
        double g = 1.0 - eps * sin2 / (1.0 + eps * eps);
        note(M_REJECT, c, g, 1.0);
        if (c <= g) break;
        if (trial == ORC_MAX_TRIALS - 1) res->reject_capped = 1;
    }
    double phi = 2.0 * ORC_PI * draw(pb, t, j);
    double up[3];
    rotate(t->u, 1.0 - omc, phi, up);
    double Ep = eps * E;
    double Te = E - Ep;
    note_rel(M_SECONDARY_CUT, Te, pb->ecut);
    note_rel(M_SECONDARY_CUT, Ep, pb->ecut);
    if (Te >= pb->ecut) {
        double ue[3] = {E * t->u[0] - Ep * up[0], E * t->u[1] - Ep * up[1], E * t->u[2] - Ep * up[2]};
        normalize(ue);
        add_secondary(res, t, ELECTRON, Te, ue, child_key(pb, t->event, t->key, t->step, 0));
    } else {
        deposit(res, Te);
    }
    if (Ep < pb->ecut) {
        deposit(res, Ep);
        t->T = 0.0;
        t->alive = 0;
    } else {
        t->T = Ep;
        memcpy(t->u, up, sizeof(up));
    }
}

static void photoelectric(const orc_problem* pb, orc_track* t, orc_step_result* res)
{
    double Te = t->T;
    note_rel(M_SECONDARY_CUT, Te, pb->ecut);
    if (Te >= pb->ecut) add_secondary(res, t, ELECTRON, Te, t->u, child_key(pb, t->event, t->key, t->step, 0));
    else deposit(res, Te);
    t->T = 0.0;
    t->alive = 0;
}

static void pair(const orc_problem* pb, orc_track* t, int* j, orc_step_result* res)
{
    double E = t->T, a = ORC_ME / E, x = 0.5;
    for (int trial = 0; trial < ORC_MAX_TRIALS; ++trial) {
        x = a + (1.0 - 2.0 * a) * draw(pb, t, j);
        double acc = draw(pb, t, j);
        note(M_REJECT, acc, 1.0 - 4.0 / 3.0 * x * (1.0 - x), 1.0);
        if (acc <= 1.0 - 4.0 / 3.0 * x * (1.0 - x)) break;
        if (trial == ORC_MAX_TRIALS - 1) res->reject_capped = 1;
    }
    double Tp = x * E - ORC_ME, Tm = (1.0 - x) * E - ORC_ME;
    note_rel(M_SECONDARY_CUT, Tm, pb->ecut);
    note_rel(M_SECONDARY_CUT, Tp, pb->ecut);
    if (Tm >= pb->ecut) add_secondary(res, t, ELECTRON, Tm, t->u, child_key(pb, t->event, t->key, t->step, 0));
    else deposit(res, Tm);
    uint64_t kp = child_key(pb, t->event, t->key, t->step, 1);
    if (Tp >= pb->ecut) {
        add_secondary(res, t, POSITRON, Tp, t->u, kp);
    } else {
        /* a positron below the cut is never tracked: it deposits its kinetic
         * energy and annihilates at the vertex with its own key at step 0 */
        deposit(res, Tp);
        annihilate(pb, t, kp, 0, res);
    }
    res->n_pair += 1;
    t->T = 0.0;
    t->alive = 0;
}

/* shared Moller/Bhabha final state for a delta ray of energy fraction eps */
static void delta_final_state(const orc_problem* pb, orc_track* t, double eps, int* j, orc_step_result* res)
{
    double T = t->T;
    double phi = 2.0 * ORC_PI * draw(pb, t, j);
    double Td = eps * T;
    double cosd = sqrt(Td * (T + 2.0 * ORC_ME) / (T * (Td + 2.0 * ORC_ME)));
    double ud[3];
    rotate(t->u, cosd, phi, ud);
    double p = sqrt(T * (T + 2.0 * ORC_ME)), pd = sqrt(Td * (Td + 2.0 * ORC_ME));
    double un[3] = {p * t->u[0] - pd * ud[0], p * t->u[1] - pd * ud[1], p * t->u[2] - pd * ud[2]};
    double Tn = T - Td;
    note_rel(M_SECONDARY_CUT, Td, pb->ecut);
    note_rel(M_SECONDARY_CUT, Tn, pb->ecut);
    if (Td >= pb->ecut) add_secondary(res, t, ELECTRON, Td, ud, child_key(pb, t->event, t->key, t->step, 0));
    else deposit(res, Td);
    if (Tn < pb->ecut) {
        t->T = Tn;
        stop_track(pb, t, res);
    } else {
        normalize(un);
        t->T = Tn;
        memcpy(t->u, un, sizeof(un));
    }
}

static void moller(const orc_problem* pb, orc_track* t, int* j, orc_step_result* res)
{
    double T = t->T, xc = pb->ecut / T;
    double g = (T + ORC_ME) / ORC_ME;
    double C1 = ((g - 1.0) / g) * ((g - 1.0) / g);
    double C2 = (2.0 * g - 1.0) / (g * g);
    double bound = 1.0 + C1 / 4.0 + fmax(0.0, 1.0 - C2);
    double eps = 0.5;
    for (int trial = 0; trial < ORC_MAX_TRIALS; ++trial) {
        eps = xc / (1.0 - draw(pb, t, j) * (1.0 - 2.0 * xc));
        double acc = draw(pb, t, j);
        double f = eps * eps * (C1 + 1.0 / (eps * eps) + 1.0 / ((1.0 - eps) * (1.0 - eps))
                                - C2 / (eps * (1.0 - eps)));
        note(M_REJECT, acc * bound, f, bound);
        if (acc * bound <= f) break;
        if (trial == ORC_MAX_TRIALS - 1) res->reject_capped = 1;
    }
    delta_final_state(pb, t, eps, j, res);
}

static void bhabha(const orc_problem* pb, orc_track* t, int* j, orc_step_result* res)
{
    double T = t->T, xc = pb->ecut / T;
    double g = (T + ORC_ME) / ORC_ME;
    double b2 = 1.0 - 1.0 / (g * g);
    double y = 1.0 / (1.0 + g);
    double B1 = 2.0 - y * y;
    double B2 = (1.0 - 2.0 * y) * (3.0 + y * y);
    double B4 = (1.0 - 2.0 * y) * (1.0 - 2.0 * y) * (1.0 - 2.0 * y);
    double B3 = B4 + (1.0 - 2.0 * y) * (1.0 - 2.0 * y);
    double eps = 0.5;
    for (int trial = 0; trial < ORC_MAX_TRIALS; ++trial) {
        eps = xc / (1.0 - draw(pb, t, j) * (1.0 - xc));
        double acc = draw(pb, t, j);
        double f = 1.0 - b2 * (B1 * eps - B2 * eps * eps + B3 * eps * eps * eps - B4 * eps * eps * eps * eps);
        note(M_REJECT, acc, f, 1.0);
        if (acc <= f) break;
        if (trial == ORC_MAX_TRIALS - 1) res->reject_capped = 1;
    }
    delta_final_state(pb, t, eps, j, res);
}

static void brems(const orc_problem* pb, orc_track* t, int* j, orc_step_result* res)
{
    double T = t->T, E = T + ORC_ME;
    double yc = pb->ecut / E, ym = T / E;
    double lr = log(ym / yc);
    double y = yc;
    for (int trial = 0; trial < ORC_MAX_TRIALS; ++trial) {
        y = yc * exp(draw(pb, t, j) * lr);
        double acc = draw(pb, t, j);
        note(M_REJECT, acc, 1.0 - y + 0.75 * y * y, 1.0);
        if (acc <= 1.0 - y + 0.75 * y * y) break;
        if (trial == ORC_MAX_TRIALS - 1) res->reject_capped = 1;
    }
    double k = y * E;
    note_rel(M_SECONDARY_CUT, k, pb->ecut);
    note_rel(M_SECONDARY_CUT, T - k, pb->ecut);
    if (k >= pb->ecut) add_secondary(res, t, GAMMA, k, t->u, child_key(pb, t->event, t->key, t->step, 0));
    else deposit(res, k);
    double Tn = T - k;
    t->T = Tn;
    if (Tn < pb->ecut) stop_track(pb, t, res);
}

/* run the final-state sampler of process `proc` at the track's current state,
 * drawing uniforms from index *j on */
void orc_interact(const orc_problem* pb, orc_track* t, int proc, int* j, orc_step_result* res)
{
    switch (proc) {
    case P_COMPTON: compton(pb, t, j, res); break;
    case P_PHOTO:   photoelectric(pb, t, res); break;
    case P_PAIR:    pair(pb, t, j, res); break;
    case P_MOLLER:  moller(pb, t, j, res); break;
    case P_BHABHA:  bhabha(pb, t, j, res); break;
    case P_BREMS:   brems(pb, t, j, res); break;
    }
}

/* ------------------------------------------------------------------ geometry */
static double zlo(const orc_problem* pb, int slab) { return pb->z_planes[slab]; }
static double zhi(const orc_problem* pb, int slab) { return pb->z_planes[slab + 1]; }

/* straight-line distance to leave the current slab box; *face gets the face */
static double straight_distance(const orc_problem* pb, const orc_track* t, int* face)
{
    double W = pb->half_width;
    double dz = INFINITY, dx = INFINITY, dy = INFINITY;
    int fz = F_NONE, fx = F_NONE, fy = F_NONE;
    note_sign(M_DIR_SIGN, t->u[0], 1.0);
    note_sign(M_DIR_SIGN, t->u[1], 1.0);
    note_sign(M_DIR_SIGN, t->u[2], 1.0);
    if (t->u[2] > 0.0) { dz = (zhi(pb, t->slab) - t->r[2]) / t->u[2]; fz = F_ZHI; }
    else if (t->u[2] < 0.0) { dz = (zlo(pb, t->slab) - t->r[2]) / t->u[2]; fz = F_ZLO; }
    if (t->u[0] > 0.0) { dx = (W - t->r[0]) / t->u[0]; fx = F_XHI; }
    else if (t->u[0] < 0.0) { dx = (-W - t->r[0]) / t->u[0]; fx = F_XLO; }
    if (t->u[1] > 0.0) { dy = (W - t->r[1]) / t->u[1]; fy = F_YHI; }
    else if (t->u[1] < 0.0) { dy = (-W - t->r[1]) / t->u[1]; fy = F_YLO; }
    dz = fmax(dz, 0.0); dx = fmax(dx, 0.0); dy = fmax(dy, 0.0);
    double d = dz;
    *face = fz;
    if (isfinite(dx) && isfinite(d)) note_rel(M_FACE_TIE, dx, d);
    if (dx < d) { d = dx; *face = fx; }
    if (isfinite(dy) && isfinite(d)) note_rel(M_FACE_TIE, dy, d);
    if (dy < d) { d = dy; *face = fy; }
    return d;
}

static double face_plane(const orc_problem* pb, int slab, int face)
{
    switch (face) {
    case F_ZLO: return zlo(pb, slab);
    case F_ZHI: return zhi(pb, slab);
    case F_XLO: return -pb->half_width;
    case F_XHI: return pb->half_width;
    case F_YLO: return -pb->half_width;
    case F_YHI: return pb->half_width;
    }
    return 0.0;
}

static int face_axis(int face) { return face == F_ZLO || face == F_ZHI ? 2 : (face <= F_XHI ? 0 : 1); }

/* one classical RK4 step of dr/ds = u, du/ds = kf (u x B) over length h */
void orc_rk4(const double r[3], const double u[3], double h, double kf, const double B[3],
             double r1[3], double u1[3])
{
#define CROSS(a, o) do { o[0] = kf * (a[1] * B[2] - a[2] * B[1]); \
                         o[1] = kf * (a[2] * B[0] - a[0] * B[2]); \
                         o[2] = kf * (a[0] * B[1] - a[1] * B[0]); } while (0)
    double k1[3], k2[3], k3[3], k4[3], u2[3], u3[3], u4[3];
    CROSS(u, k1);
    for (int c = 0; c < 3; ++c) u2[c] = u[c] + 0.5 * h * k1[c];
    CROSS(u2, k2);
    for (int c = 0; c < 3; ++c) u3[c] = u[c] + 0.5 * h * k2[c];
    CROSS(u3, k3);
    for (int c = 0; c < 3; ++c) u4[c] = u[c] + h * k3[c];
    CROSS(u4, k4);
    for (int c = 0; c < 3; ++c) {
        r1[c] = r[c] + h / 6.0 * (u[c] + 2.0 * u2[c] + 2.0 * u3[c] + u4[c]);
        u1[c] = u[c] + h / 6.0 * (k1[c] + 2.0 * k2[c] + 2.0 * k3[c] + k4[c]);
    }
#undef CROSS
}

/* first face of the slab box that the chord r -> r1 crosses; *f = chord fraction */
static int chord_crossing(const orc_problem* pb, int slab, const double r[3], const double r1[3], double* f)
{
    double W = pb->half_width;
    int best = F_NONE;
    double bf = INFINITY;
    for (int face = F_ZLO; face <= F_YHI; ++face) {
        int ax = face_axis(face);
        double p = face_plane(pb, slab, face);
        int beyond = (face == F_ZLO || face == F_XLO || face == F_YLO) ? (r1[ax] < p) : (r1[ax] > p);
        note(M_CHORD_BEYOND, r1[ax], p, fmax(fabs(p), 1.0));
        if (!beyond) continue;
        double fr = (p - r[ax]) / (r1[ax] - r[ax]);
        note_sign(M_CHORD_AT_START, fr, 1.0);
        if (fr < 0.0) fr = 0.0;
        if (fr > 1.0) fr = 1.0;
        if (isfinite(bf)) note(M_CHORD_FACE_TIE, fr, bf, 1.0);
        if (fr < bf) { bf = fr; best = face; }
    }
    (void)W;
    *f = bf;
    return best;
}

/* does direction u point out of the box through `face`? */
static int points_out(const double u[3], int face)
{
    switch (face) {
    case F_ZLO: return u[2] < 0.0;
    case F_ZHI: return u[2] > 0.0;
    case F_XLO: return u[0] < 0.0;
    case F_XHI: return u[0] > 0.0;
    case F_YLO: return u[1] < 0.0;
    case F_YHI: return u[1] > 0.0;
    }
    return 0;
}

/* face of the slab box nearest to point r within the search tolerance, or F_NONE */
static int near_face(const orc_problem* pb, int slab, const double r[3])
{
    int best = F_NONE;
    double bd = ORC_DINT;
    for (int face = F_ZLO; face <= F_YHI; ++face) {
        double d = fabs(r[face_axis(face)] - face_plane(pb, slab, face));
        note(M_NEAR_FACE, d, bd, ORC_DINT);
        if (d <= bd && (best == F_NONE || d < bd)) { bd = d; best = face; }
    }
    return best;
}

/* Field propagation of a charged track over at most s_phys (momentum fixed).
 * Substep h = min(remaining, sqrt(8 d_chord / curvature)), one classical RK4
 * each, direction renormalised after every accepted substep.  When the chord
 * of a substep leaves the slab box, the substep is retried from its start with
 * h scaled by the chord fraction at the crossed plane (halved when the chord
 * leaves at its very start while the tangent points inward) until the chord
 * overshoot or the retried end point is within d_int of the plane, or 10
 * retries; the crossing point is then snapped onto the plane.
 * Returns the path length; *face is the crossed face or F_NONE. */
double orc_propagate_field(const orc_problem* pb, orc_track* t, double s_phys, int* face, int* n_substeps)
{
    double q = t->type == POSITRON ? 1.0 : -1.0;
    double p = sqrt(t->T * (t->T + 2.0 * ORC_ME));
    double kf = q * ORC_CK / p;
    double Bm = sqrt(pb->B[0] * pb->B[0] + pb->B[1] * pb->B[1] + pb->B[2] * pb->B[2]);
    double kappa = ORC_CK * Bm / p;
    double h_chord = sqrt(8.0 * ORC_DCHORD / kappa);
    double s_done = 0.0, h_try = 0.0;
    int n_search = 0, count = 0;
    *face = F_NONE;
    for (;;) {
        double rem = s_phys - s_done;
        double h = h_try > 0.0 ? h_try : fmin(rem, h_chord);
        if (h_try == 0.0) note_rel(M_LAST_SUBSTEP, rem, h_chord);
        int last = (h_try == 0.0 && h == rem);
        double r1[3], u1[3];
        orc_rk4(t->r, t->u, h, kf, pb->B, r1, u1);
        count += 1;
        double f;
        int fc = chord_crossing(pb, t->slab, t->r, r1, &f);
        if (fc == F_NONE) {
            int nf = h_try > 0.0 ? near_face(pb, t->slab, r1) : F_NONE;
            memcpy(t->r, r1, sizeof(r1));
            normalize(u1);
            memcpy(t->u, u1, sizeof(u1));
            if (nf != F_NONE) {
                t->r[face_axis(nf)] = face_plane(pb, t->slab, nf);
                s_done += h;
                *face = nf;
                break;
            }
            if (last) { s_done = s_phys; break; }
            s_done += h;
            h_try = 0.0;
            n_search = 0;
            continue;
        }
        if (f == 0.0) note_sign(M_DIR_SIGN, t->u[face_axis(fc)], 1.0);
        if (f == 0.0 && points_out(t->u, fc)) {
            /* already on the plane and heading out: leave without moving */
            t->r[face_axis(fc)] = face_plane(pb, t->slab, fc);
            *face = fc;
            break;
        }
        double ch[3] = {r1[0] - t->r[0], r1[1] - t->r[1], r1[2] - t->r[2]};
        double clen = sqrt(ch[0] * ch[0] + ch[1] * ch[1] + ch[2] * ch[2]);
        if (n_search < ORC_MAX_SEARCH) note(M_SEARCH_ACCEPT, (1.0 - f) * clen, ORC_DINT, ORC_DINT);
        if ((1.0 - f) * clen <= ORC_DINT || n_search >= ORC_MAX_SEARCH) {
            for (int c = 0; c < 3; ++c) t->r[c] = t->r[c] + f * ch[c];
            t->r[face_axis(fc)] = face_plane(pb, t->slab, fc);
            normalize(u1);
            memcpy(t->u, u1, sizeof(u1));
            s_done += f * h;
            *face = fc;
            break;
        }
        h_try = f > 0.0 ? f * h : 0.5 * h;
        n_search += 1;
    }
    if (n_substeps) *n_substeps = count;
    return s_done;
}

static int has_field(const orc_problem* pb) { return pb->B[0] != 0.0 || pb->B[1] != 0.0 || pb->B[2] != 0.0; }

/* ------------------------------------------------------------------ one step */
/* ------------------------------------------------------------------ multiple scattering
 * Optional angular deflection of charged tracks after each along-step (no
 * lateral displacement).  The projected scattering angles are taken as
 * Gaussian with the Highland width (PDG review of particle properties,
 * "Passage of particles through matter", multiple scattering through small
 * angles) for a singly charged particle:
 *     theta0 = 13.6 MeV / (beta c p) * sqrt(x) * (1 + 0.038 ln(x / beta^2)),
 *     x = s / X0,
 * at the pre-step kinetic energy.  Two independent Gaussian projections make
 * the space angle Rayleigh distributed: theta = theta0 sqrt(-2 ln U_a), with
 * a uniform azimuth 2 pi U_b.  U_a, U_b are words 0 and 1 of the Philox block
 * at counter (key, step, 0, 5).  No deflection when s = 0 or when the bracket
 * is not positive (x / beta^2 below about 4e-12). */
double orc_msc_theta0(double T, double s, double X0)
{
    if (!(s > 0.0)) return 0.0;
    double p = sqrt(T * (T + 2.0 * ORC_ME));
    double beta = p / (T + ORC_ME);
    double x = s / X0;
    double bracket = 1.0 + 0.038 * log(x / (beta * beta));
    if (!(bracket > 0.0)) return 0.0;
    return 13.6 / (beta * p) * sqrt(x) * bracket;
}

static void msc_deflect(const orc_problem* pb, orc_track* t, int mat, double T_pre, double s)
{
    double theta0 = orc_msc_theta0(T_pre, s, pb->x0_cm[mat]);
    if (theta0 == 0.0) return;
    double ua = to_unit(philox_word(pb, t->event, t->key, t->step, 0, 5, 0));
    double ub = to_unit(philox_word(pb, t->event, t->key, t->step, 0, 5, 1));
    double theta = theta0 * sqrt(-2.0 * log(ua));
    double out[3];
    rotate(t->u, cos(theta), 2.0 * ORC_PI * ub, out);
    normalize(out);
    t->u[0] = out[0]; t->u[1] = out[1]; t->u[2] = out[2];
}

/* test hook: deflect t (material mat, pre-step energy T_pre, step s) */
void orc_msc_deflect(const orc_problem* pb, orc_track* t, int mat, double T_pre, double s)
{
    msc_deflect(pb, t, mat, T_pre, s);
}

void orc_step(const orc_problem* pb, orc_track* t, orc_step_result* res)
{
    memset(res, 0, sizeof(*res));
    res->process = -1;
    res->dep_slab = t->slab;
    int mat = pb->slab_material[t->slab];
    int charged = t->type != GAMMA;
    int j = 0;

    /* a track below the tracking cut is stopped at the start of its step */
    note_rel(M_CUT_START, t->T, pb->ecut);
    if (t->T < pb->ecut) {
        if (charged) stop_track(pb, t, res);
        else { deposit(res, t->T); t->T = 0.0; t->alive = 0; }
        res->outcome = OUT_STOP;
        t->step += 1;
        return;
    }

    const double T_pre = t->T;
    /* S1 */
    if (t->nl < 0.0) {
        t->nl = -log(draw(pb, t, &j));
        res->drew_u0 = 1;
    }
    /* S2 */
    double sig = total_xs(pb, mat, t->type, t->T);
    double s_int = sig > 0.0 ? t->nl / sig : INFINITY;
    /* S3 */
    double s_phys = s_int, R = 0.0;
    int loss_limited = 0;
    if (charged) {
        R = lookup(range_tab(pb, mat, t->type), t->T);
        double s_loss = R <= ORC_R_FINAL ? R : fmax(ORC_R_FINAL, ORC_RHO_RANGE * R);
        if (isfinite(s_int)) note_rel(M_LOSS_VS_INT, s_loss, s_int);
        if (s_loss < s_int) { s_phys = s_loss; loss_limited = 1; }
    }
    /* S4, S5 */
    double s;
    int face = F_NONE;
    if (!charged || !has_field(pb)) {
        double s_geo = straight_distance(pb, t, &face);
        if (isfinite(s_geo) && isfinite(s_phys)) note_rel(M_GEO_VS_PHYS, s_geo, s_phys);
        if (s_geo <= s_phys) s = s_geo;
        else { s = s_phys; face = F_NONE; }
        for (int c = 0; c < 3; ++c) t->r[c] = t->r[c] + s * t->u[c];
        if (face != F_NONE) t->r[face_axis(face)] = face_plane(pb, t->slab, face);
    } else {
        s = orc_propagate_field(pb, t, s_phys, &face, NULL);
    }
    res->step_len = s;
    res->face = face;

    /* S6 */
    if (charged) {
        if (face == F_NONE && loss_limited) note_rel(M_RANGE_FINAL, R, ORC_R_FINAL);
        if (face == F_NONE && loss_limited && R <= ORC_R_FINAL) {
            stop_track(pb, t, res);
            res->outcome = OUT_STOP;
            t->step += 1;
            return;
        }
        double Tn = inverse_range(range_tab(pb, mat, t->type), R - s);
        note_rel(M_CUT_AFTER_LOSS, Tn, pb->ecut);
        if (Tn < pb->ecut) {
            stop_track(pb, t, res);
            res->outcome = OUT_STOP;
            t->step += 1;
            return;
        }
        deposit(res, t->T - Tn);
        t->T = Tn;
    }
    /* S7 */
    t->nl = t->nl - s * sig;
    /* S7b: not for a track leaving the stack */
    if (charged && pb->msc) {
        int leaving = 0;
        if (face != F_NONE) {
            int next = face == F_ZLO ? t->slab - 1 : (face == F_ZHI ? t->slab + 1 : -1);
            leaving = next < 0 || next >= pb->n_slabs;
        }
        if (!leaving) msc_deflect(pb, t, mat, T_pre, s);
    }

    /* S8, S9 */
    if (face != F_NONE) {
        int next = t->slab;
        if (face == F_ZLO) next = t->slab - 1;
        else if (face == F_ZHI) next = t->slab + 1;
        else next = -1;
        if (next < 0 || next >= pb->n_slabs) {
            res->escaped = t->T;
            res->outcome = OUT_ESCAPE;
            t->T = 0.0;
            t->alive = 0;
        } else {
            t->slab = next;
            res->outcome = OUT_BOUNDARY;
        }
    } else if (loss_limited) {
        res->outcome = OUT_LOSS;
    } else {
        double U1 = draw(pb, t, &j);
        double sig1 = total_xs(pb, mat, t->type, t->T);
        t->nl = -1.0;
        if (sig1 > 0.0) {
            double target = U1 * sig1, cum = 0.0;
            int proc = proc_of(t->type, n_procs(t->type) - 1);
            for (int n = 0; n < n_procs(t->type); ++n) {
                cum += xs(pb, mat, proc_of(t->type, n), t->T);
                if (n < n_procs(t->type) - 1) note(M_PROCESS, target, cum, sig1);
                if (target < cum) { proc = proc_of(t->type, n); break; }
            }
            res->process = proc;
            res->outcome = OUT_INTERACT;
            orc_interact(pb, t, proc, &j, res);
        } else {
            res->outcome = OUT_NO_INTERACT;
        }
    }
    res->n_draws = j;
    /* S10 */
    t->step += 1;
    if (t->alive && t->step > ORC_MAX_STEPS) {
        if (charged) stop_track(pb, t, res);
        else { deposit(res, t->T); t->T = 0.0; t->alive = 0; }
        res->outcome = OUT_GUARD;
    }
}

/* ------------------------------------------------------------------ events */
typedef struct {
    orc_track* v;
    size_t n, cap;
} stack_t_;

static void push(stack_t_* s, const orc_track* t)
{
    if (s->n == s->cap) {
        s->cap = s->cap ? 2 * s->cap : 256;
        s->v = (orc_track*)realloc(s->v, s->cap * sizeof(orc_track));
    }
    s->v[s->n++] = *t;
}

/* transport every primary of one event to completion, LIFO over secondaries */
static uint64_t run_one_event(const orc_problem* pb, const orc_track* prims, const uint64_t* idx, uint64_t n,
                              double* edep, orc_ledger* led)
{
    stack_t_ st = {0, 0, 0};
    for (uint64_t i = 0; i < n; ++i) push(&st, &prims[idx[i]]);
    uint64_t steps = 0;
    orc_step_result res;
    while (st.n > 0) {
        orc_track t = st.v[--st.n];
        t.alive = 1;
        while (t.alive) {
            orc_step(pb, &t, &res);
            steps += 1;
            edep[res.dep_slab] += res.edep;
            led->escaped += res.escaped;
            led->n_pair += (uint64_t)res.n_pair;
            led->n_annih += (uint64_t)res.n_annih;
            led->n_reject_cap += (uint64_t)res.reject_capped;
            if (res.outcome == OUT_GUARD) led->n_guard += 1;
            for (int k = 0; k < res.n_sec; ++k) {
                led->n_sec[res.sec[k].type] += 1;
                push(&st, &res.sec[k]);
            }
        }
    }
    led->steps += steps;
    free(st.v);
    return steps;
}

typedef struct {
    const orc_problem* pb;
    const orc_track* prims;
    const uint64_t* order;     /* primaries sorted by row */
    const uint64_t* row_start; /* n_rows + 1 */
    uint32_t n_rows;
    double* edep;
    orc_ledger* ledger;
    int tid, nthreads;
    uint64_t steps;
} worker_arg;

static void* worker(void* p)
{
    worker_arg* a = (worker_arg*)p;
    a->steps = 0;
    for (uint32_t row = (uint32_t)a->tid; row < a->n_rows; row += (uint32_t)a->nthreads) {
        uint64_t b = a->row_start[row], e = a->row_start[row + 1];
        a->steps += run_one_event(a->pb, a->prims, a->order + b, e - b,
                                  a->edep + (size_t)row * (size_t)a->pb->n_slabs, &a->ledger[row]);
    }
    return NULL;
}

/* Transport all primaries; prim_row[i] is the tally row of primary i.
 * edep: [n_rows][n_slabs] (zeroed here); ledger: [n_rows].  Rows are spread
 * over n_threads POSIX threads; each event runs sequentially, so results do
 * not depend on the thread count.  Returns the number of steps taken. */
uint64_t orc_run_events(const orc_problem* pb, const orc_track* prims, const uint32_t* prim_row, uint64_t n_prim,
                        uint32_t n_rows, double* edep, orc_ledger* ledger, int n_threads)
{
    memset(edep, 0, sizeof(double) * (size_t)n_rows * (size_t)pb->n_slabs);
    memset(ledger, 0, sizeof(orc_ledger) * n_rows);
    uint64_t* row_start = (uint64_t*)calloc((size_t)n_rows + 1, sizeof(uint64_t));
    uint64_t* order = (uint64_t*)malloc(sizeof(uint64_t) * (n_prim ? n_prim : 1));
    for (uint64_t i = 0; i < n_prim; ++i) row_start[prim_row[i] + 1] += 1;
    for (uint32_t r = 0; r < n_rows; ++r) row_start[r + 1] += row_start[r];
    uint64_t* fill = (uint64_t*)malloc(sizeof(uint64_t) * ((size_t)n_rows + 1));
    memcpy(fill, row_start, sizeof(uint64_t) * ((size_t)n_rows + 1));
    for (uint64_t i = 0; i < n_prim; ++i) order[fill[prim_row[i]]++] = i;
    free(fill);

    if (n_threads < 1) n_threads = 1;
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)n_threads);
    worker_arg* args = (worker_arg*)malloc(sizeof(worker_arg) * (size_t)n_threads);
    for (int i = 0; i < n_threads; ++i) {
        args[i] = (worker_arg){pb, prims, order, row_start, n_rows, edep, ledger, i, n_threads, 0};
        pthread_create(&th[i], NULL, worker, &args[i]);
    }
    uint64_t steps = 0;
    for (int i = 0; i < n_threads; ++i) {
        pthread_join(th[i], NULL);
        steps += args[i].steps;
    }
    free(th);
    free(args);
    free(order);
    free(row_start);
    return steps;
}

/* ------------------------------------------------------------------ flip diagnosis
 * One step with its decision margins recorded (see note()). */
void orc_step_margin(const orc_problem* pb, orc_track* t, orc_step_result* res, orc_margin* m)
{
    m->margin = INFINITY;
    m->kind = M_NONE;
    m->n_notes = 0;
    g_margin = m;
    orc_step(pb, t, res);
    g_margin = NULL;
}

/* one recorded step of an event history: the track before and after it, the
 * step's result and the smallest decision margin of the step */
typedef struct {
    orc_track pre;
    orc_track post;
    orc_step_result res;
    orc_margin m;
} orc_trace_rec;

/* Transport the n primaries of one event exactly as orc_run_events does (LIFO
 * over secondaries) and record every step in history order: a step's
 * ancestors (its track's earlier steps, the step that created the track)
 * always come before it.  Writes up to `cap` records and returns the number
 * of steps. */
uint64_t orc_trace_event(const orc_problem* pb, const orc_track* prims, uint64_t n, orc_trace_rec* out, uint64_t cap)
{
    stack_t_ st = {0, 0, 0};
    for (uint64_t i = 0; i < n; ++i) push(&st, &prims[i]);
    uint64_t steps = 0;
    orc_trace_rec rec;
    while (st.n > 0) {
        orc_track t = st.v[--st.n];
        t.alive = 1;
        while (t.alive) {
            rec.pre = t;
            orc_step_margin(pb, &t, &rec.res, &rec.m);
            rec.post = t;
            if (steps < cap) out[steps] = rec;
            steps += 1;
            for (int k = 0; k < rec.res.n_sec; ++k) push(&st, &rec.res.sec[k]);
        }
    }
    free(st.v);
    return steps;
}

/* table lookups exposed for the pins */
double orc_lookup(const double* v, double T) { return lookup(v, T); }
double orc_inverse_range(const double* R, double r) { return inverse_range(R, r); }
double orc_xs(const orc_problem* pb, int mat, int proc, double T) { return xs(pb, mat, proc, T); }
