// Device physics of the electromagnetic step loop: table interpolation,
// process cross sections, final-state samplers and annihilation at rest.
//
// The paper (arXiv 2503.17608) states only that the transport covers EM
// processes of photons, electrons and positrons.  The models used are named
// textbook forms: Klein-Nishina Compton with Butcher-Messel sampling, Born
// K-shell photoelectric (x 5/4), complete-screening Bethe-Heitler pair
// production, Moller and Bhabha delta rays above the cut, Tsai complete-
// screening bremsstrahlung above the cut, restricted continuous loss through
// a range table, annihilation at rest into two back-to-back photons.
//
// Template parameter R is the precision of energies, directions, cross
// sections and tables (double, or float in the mixed mode); positions and
// path lengths are always double.
#pragma once
#include "common.hpp"

namespace ems {

template <class R>
struct Tables {
    const R* v;        // [n_mat][8][181]
    R ln_e0;
    R inv_dlog;
    R dlog;
    __device__ __forceinline__ const R* tab(int mat, int which) const
    {
        return v + (mat * kTabPerMat + which) * kNodes;
    }
};

// interpolation location of energy T on the log grid
template <class R>
struct Loc {
    int i;
    R f;
};

template <class R>
__device__ __forceinline__ Loc<R> locate(const Tables<R>& tb, R T)
{
    R t = (m_log(T) - tb.ln_e0) * tb.inv_dlog;
    R fl = m_floor(t);
    int i = (int)fl;
    if (fl < R(0)) i = 0;
    if (fl > R(kNodes - 2)) i = kNodes - 2;
    Loc<R> l;
    l.i = i;
    l.f = t - R(i);
    return l;
}

template <class R>
__device__ __forceinline__ R interp(const R* v, const Loc<R>& l)
{
    R a = v[l.i], b = v[l.i + 1];
    return a + l.f * (b - a);
}

// macroscopic cross section of process p at T, zero at and below its threshold
template <class R>
__device__ __forceinline__ R proc_xs(const Tables<R>& tb, int mat, int p, R T, const Loc<R>& l, R ecut)
{
    switch (p) {
    case P_COMPTON: return interp(tb.tab(mat, TB_COMPTON), l);
    case P_PHOTO:   return interp(tb.tab(mat, TB_PHOTO), l);
    case P_PAIR:    return T <= R(2.0 * kMe) ? R(0) : interp(tb.tab(mat, TB_PAIR), l);
    case P_MOLLER:  return T <= R(2) * ecut ? R(0) : interp(tb.tab(mat, TB_MOLLER), l);
    case P_BHABHA:  return T <= ecut ? R(0) : interp(tb.tab(mat, TB_BHABHA), l);
    default:        return T <= ecut ? R(0) : interp(tb.tab(mat, TB_BREMS), l);
    }
}

// processes of each particle, in selection order
__device__ __forceinline__ int n_proc(int type) { return type == kGamma ? 3 : 2; }
__device__ __forceinline__ int proc_of(int type, int n)
{
    if (type == kGamma) return n;                       // Compton, photoelectric, pair
    if (type == kElectron) return n == 0 ? P_MOLLER : P_BREMS;
    return n == 0 ? P_BHABHA : P_BREMS;
}

template <class R>
__device__ __forceinline__ R total_xs(const Tables<R>& tb, int mat, int type, R T, const Loc<R>& l, R ecut)
{
    R s = R(0);
    for (int n = 0; n < n_proc(type); ++n) s += proc_xs(tb, mat, proc_of(type, n), T, l, ecut);
    return s;
}

template <class R>
__device__ __forceinline__ const R* range_tab(const Tables<R>& tb, int mat, int type)
{
    return tb.tab(mat, type == kPositron ? TB_RANGE_EP : TB_RANGE_EM);
}

// Exact inverse of the piecewise-linear range map: the interval is the one an
// upper-bound search on the node ranges finds (first node with R > r, minus
// one); ln T is linear in R inside it.  The search walks down from a starting
// node `j0` (the interval of the pre-step energy, since r <= R(T)), which
// finds the same interval as a binary search in one or two probes.
template <class R>
__device__ __forceinline__ R inverse_range(const Tables<R>& tb, const R* Rt, R r, int j0)
{
    int j = j0 < kNodes ? j0 : kNodes;
    while (j < kNodes && !(Rt[j] > r)) ++j;
    while (j > 0 && Rt[j - 1] > r) --j;
    int i = j - 1;
    if (i < 0) i = 0;
    if (i > kNodes - 2) i = kNodes - 2;
    R t = R(i) + (r - Rt[i]) / (Rt[i + 1] - Rt[i]);
    return m_exp(tb.ln_e0 + t * tb.dlog);
}

// rotate direction u by polar cosine c and azimuth phi (phi given as sin/cos)
template <class R>
__device__ __forceinline__ void rotate(const R u[3], R c, R sp, R cp, R out[3])
{
    if (c > R(1)) c = R(1);
    if (c < R(-1)) c = R(-1);
    R s = m_sqrt(R(1) - c * c);
    R a = m_sqrt(R(1) - u[2] * u[2]);
    if (a > R(1.0e-10)) {
        out[0] = u[0] * c + s * (u[0] * u[2] * cp - u[1] * sp) / a;
        out[1] = u[1] * c + s * (u[1] * u[2] * cp + u[0] * sp) / a;
        out[2] = u[2] * c - a * s * cp;
    } else {
        out[0] = s * cp;
        out[1] = s * sp;
        out[2] = (u[2] >= R(0) ? R(1) : R(-1)) * c;
    }
}

template <class R>
__device__ __forceinline__ void normalize3(R v[3])
{
    R n = m_sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    v[0] /= n; v[1] /= n; v[2] /= n;
}

// up to three secondaries produced by one track step, kept in registers
// (fixed slots, selected with compile-time indices after unrolling)
template <class R>
struct Sec {
    R T;
    R ux, uy, uz;       // scalars, not an array: the buffer must stay in registers
    uint64_t key;
    int type;
};

template <class R>
struct SecBuf {
    int n;
    Sec<R> s0, s1, s2;
    // every field of every slot is written through a value select: branches
    // or whole-struct copies chosen at run time would be merged into stores
    // through a selected pointer, which puts the buffer on the stack
    __device__ __forceinline__ static void put(Sec<R>& s, bool here, int t, R e, const R d[3], uint64_t k)
    {
        s.T = here ? e : s.T;
        s.ux = here ? d[0] : s.ux;
        s.uy = here ? d[1] : s.uy;
        s.uz = here ? d[2] : s.uz;
        s.key = here ? k : s.key;
        s.type = here ? t : s.type;
    }
    __device__ __forceinline__ void add(int t, R e, const R d[3], uint64_t k)
    {
        put(s0, n == 0, t, e, d, k);
        put(s1, n == 1, t, e, d, k);
        put(s2, n >= 2, t, e, d, k);
        ++n;
    }
    // Visit the stored secondaries in order, by name (no run-time index, so
    // the buffer stays in registers): f(secondary, ordinal).
    template <class F>
    __device__ __forceinline__ void each(F&& f) const
    {
        if (n > 0) f(s0, 0);
        if (n > 1) f(s1, 1);
        if (n > 2) f(s2, 2);
    }
};

// per-step tallies of one track
struct StepTally {
    double edep;
    int n_pair, n_annih, capped;
};

struct PhysParams {
    uint64_t seed;
    uint64_t event;    // Philox key word 1 of the track's event
    double ecut;
};

// annihilation at rest of a positron with key `key` in step `step`: two
// photons of m c^2, back to back, isotropic (Philox domain 4, block 0);
// deposited locally when m c^2 is below the cut
template <class R>
__device__ __forceinline__ void annihilate(const PhysParams& pp, uint64_t key, uint64_t step, SecBuf<R>& sb, StepTally& tl)
{
    tl.n_annih += 1;
    if (kMe < pp.ecut) {
        tl.edep += 2.0 * kMe;
        return;
    }
    U64x4 w = philox4x64_10(key, step, 0, 4, pp.seed, pp.event);
    R cost = R(2) * unit_from<R>(w.w[0]) - R(1);
    R phi = R(2.0 * kPi) * unit_from<R>(w.w[1]);
    R sp, cp;
    m_sincos(phi, &sp, &cp);
    R sint = m_sqrt(R(1) - cost * cost);
    R v[3] = {sint * cp, sint * sp, cost};
    R mv[3] = {-v[0], -v[1], -v[2]};
    sb.add(kGamma, R(kMe), v, child_key(pp.seed, pp.event, key, step, 2));
    sb.add(kGamma, R(kMe), mv, child_key(pp.seed, pp.event, key, step, 3));
}

// in/out state of the interacting track
template <class R>
struct Prim {
    R T;
    R u[3];
    uint64_t key;
    uint32_t step;
    int type;
    bool alive;
};

// the lepton stops: deposit its kinetic energy; positrons annihilate
template <class R>
__device__ __forceinline__ void stop_lepton(const PhysParams& pp, Prim<R>& t, SecBuf<R>& sb, StepTally& tl)
{
    tl.edep += (double)t.T;
    if (t.type == kPositron) annihilate<R>(pp, t.key, t.step, sb, tl);
    t.T = R(0);
    t.alive = false;
}

template <class R>
__device__ __forceinline__ void sample_compton(const PhysParams& pp, Prim<R>& t, StepRng<R>& rng, SecBuf<R>& sb, StepTally& tl)
{
    const R ec = R(pp.ecut);
    R E = t.T, kap = E / R(kMe);
    R e0 = R(1) / (R(1) + R(2) * kap), e0sq = e0 * e0;
    R a1 = -m_log(e0), a2 = R(0.5) * (R(1) - e0sq);
    R eps = R(1), omc = R(0);
    for (int trial = 0; trial < kMaxTrials; ++trial) {
        R a = rng.next(), b = rng.next(), c = rng.next();
        if (a * (a1 + a2) < a1) eps = m_exp(-a1 * b);
        else eps = m_sqrt(e0sq + (R(1) - e0sq) * b);
        omc = (R(1) - eps) / (kap * eps);
        R sin2 = omc * (R(2) - omc);
        R g = R(1) - eps * sin2 / (R(1) + eps * eps);
        if (c <= g) break;
        if (trial == kMaxTrials - 1) tl.capped = 1;
    }
    R phi = R(2.0 * kPi) * rng.next();
    R sp, cp;
    m_sincos(phi, &sp, &cp);
    R up[3];
    rotate<R>(t.u, R(1) - omc, sp, cp, up);
    R Ep = eps * E;
    R Te = E - Ep;
    if (Te >= ec) {
        R ue[3] = {E * t.u[0] - Ep * up[0], E * t.u[1] - Ep * up[1], E * t.u[2] - Ep * up[2]};
        normalize3(ue);
        sb.add(kElectron, Te, ue, child_key(pp.seed, pp.event, t.key, t.step, 0));
    } else {
        tl.edep += (double)Te;
    }
    if (Ep < ec) {
        tl.edep += (double)Ep;
        t.T = R(0);
        t.alive = false;
    } else {
        t.T = Ep;
        t.u[0] = up[0]; t.u[1] = up[1]; t.u[2] = up[2];
    }
}

template <class R>
__device__ __forceinline__ void sample_photo(const PhysParams& pp, Prim<R>& t, SecBuf<R>& sb, StepTally& tl)
{
    R Te = t.T;
    if (Te >= R(pp.ecut)) sb.add(kElectron, Te, t.u, child_key(pp.seed, pp.event, t.key, t.step, 0));
    else tl.edep += (double)Te;
    t.T = R(0);
    t.alive = false;
}

template <class R>
__device__ __forceinline__ void sample_pair(const PhysParams& pp, Prim<R>& t, StepRng<R>& rng, SecBuf<R>& sb, StepTally& tl)
{
    const R ec = R(pp.ecut);
    R E = t.T, a = R(kMe) / E, x = R(0.5);
    for (int trial = 0; trial < kMaxTrials; ++trial) {
        x = a + (R(1) - R(2) * a) * rng.next();
        R acc = rng.next();
        if (acc <= R(1) - R(4) / R(3) * x * (R(1) - x)) break;
        if (trial == kMaxTrials - 1) tl.capped = 1;
    }
    R Tp = x * E - R(kMe), Tm = (R(1) - x) * E - R(kMe);
    if (Tm >= ec) sb.add(kElectron, Tm, t.u, child_key(pp.seed, pp.event, t.key, t.step, 0));
    else tl.edep += (double)Tm;
    uint64_t kp = child_key(pp.seed, pp.event, t.key, t.step, 1);
    if (Tp >= ec) {
        sb.add(kPositron, Tp, t.u, kp);
    } else {
        // a positron below the cut is not tracked: it deposits and annihilates
        // at the vertex with its own key at step 0
        tl.edep += (double)Tp;
        annihilate<R>(pp, kp, 0, sb, tl);
    }
    tl.n_pair += 1;
    t.T = R(0);
    t.alive = false;
}

template <class R>
__device__ __forceinline__ void delta_final(const PhysParams& pp, Prim<R>& t, R eps, StepRng<R>& rng, SecBuf<R>& sb, StepTally& tl)
{
    const R ec = R(pp.ecut);
    R T = t.T;
    R phi = R(2.0 * kPi) * rng.next();
    R sp, cp;
    m_sincos(phi, &sp, &cp);
    R Td = eps * T;
    R cosd = m_sqrt(Td * (T + R(2.0 * kMe)) / (T * (Td + R(2.0 * kMe))));
    R ud[3];
    rotate<R>(t.u, cosd, sp, cp, ud);
    R p = m_sqrt(T * (T + R(2.0 * kMe))), pd = m_sqrt(Td * (Td + R(2.0 * kMe)));
    R un[3] = {p * t.u[0] - pd * ud[0], p * t.u[1] - pd * ud[1], p * t.u[2] - pd * ud[2]};
    R Tn = T - Td;
    if (Td >= ec) sb.add(kElectron, Td, ud, child_key(pp.seed, pp.event, t.key, t.step, 0));
    else tl.edep += (double)Td;
    t.T = Tn;
    if (Tn < ec) {
        stop_lepton<R>(pp, t, sb, tl);
    } else {
        normalize3(un);
        t.u[0] = un[0]; t.u[1] = un[1]; t.u[2] = un[2];
    }
}

template <class R>
__device__ __forceinline__ void sample_moller(const PhysParams& pp, Prim<R>& t, StepRng<R>& rng, SecBuf<R>& sb, StepTally& tl)
{
    R T = t.T, xc = R(pp.ecut) / T;
    R g = (T + R(kMe)) / R(kMe);
    R C1 = ((g - R(1)) / g) * ((g - R(1)) / g);
    R C2 = (R(2) * g - R(1)) / (g * g);
    R bound = R(1) + C1 / R(4) + m_max(R(0), R(1) - C2);
    R eps = R(0.5);
    for (int trial = 0; trial < kMaxTrials; ++trial) {
        eps = xc / (R(1) - rng.next() * (R(1) - R(2) * xc));
        R acc = rng.next();
        R f = eps * eps * (C1 + R(1) / (eps * eps) + R(1) / ((R(1) - eps) * (R(1) - eps)) - C2 / (eps * (R(1) - eps)));
        if (acc * bound <= f) break;
        if (trial == kMaxTrials - 1) tl.capped = 1;
    }
    delta_final<R>(pp, t, eps, rng, sb, tl);
}

template <class R>
__device__ __forceinline__ void sample_bhabha(const PhysParams& pp, Prim<R>& t, StepRng<R>& rng, SecBuf<R>& sb, StepTally& tl)
{
    R T = t.T, xc = R(pp.ecut) / T;
    R g = (T + R(kMe)) / R(kMe);
    R b2 = R(1) - R(1) / (g * g);
    R y = R(1) / (R(1) + g);
    R B1 = R(2) - y * y;
    R B2 = (R(1) - R(2) * y) * (R(3) + y * y);
    R B4 = (R(1) - R(2) * y) * (R(1) - R(2) * y) * (R(1) - R(2) * y);
    R B3 = B4 + (R(1) - R(2) * y) * (R(1) - R(2) * y);
    R eps = R(0.5);
    for (int trial = 0; trial < kMaxTrials; ++trial) {
        eps = xc / (R(1) - rng.next() * (R(1) - xc));
        R acc = rng.next();
        R f = R(1) - b2 * (B1 * eps - B2 * eps * eps + B3 * eps * eps * eps - B4 * eps * eps * eps * eps);
        if (acc <= f) break;
        if (trial == kMaxTrials - 1) tl.capped = 1;
    }
    delta_final<R>(pp, t, eps, rng, sb, tl);
}

template <class R>
__device__ __forceinline__ void sample_brems(const PhysParams& pp, Prim<R>& t, StepRng<R>& rng, SecBuf<R>& sb, StepTally& tl)
{
    const R ec = R(pp.ecut);
    R T = t.T, E = T + R(kMe);
    R yc = ec / E, ym = T / E;
    R lr = m_log(ym / yc);
    R y = yc;
    for (int trial = 0; trial < kMaxTrials; ++trial) {
        y = yc * m_exp(rng.next() * lr);
        R acc = rng.next();
        if (acc <= R(1) - y + R(0.75) * y * y) break;
        if (trial == kMaxTrials - 1) tl.capped = 1;
    }
    R k = y * E;
    if (k >= ec) sb.add(kGamma, k, t.u, child_key(pp.seed, pp.event, t.key, t.step, 0));
    else tl.edep += (double)k;
    R Tn = T - k;
    t.T = Tn;
    if (Tn < ec) stop_lepton<R>(pp, t, sb, tl);
}

}  // namespace ems
