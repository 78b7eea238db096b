/*
 * hf_oracle.c -- plain FP64 CPU oracle for the cut chain, survivor
 * compaction, adaptive cut ordering, dileptonic ttbar reconstruction and
 * the single-neutrino chi^2 reconstruction.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header or constant table with the GPU library; it is deliberately slow and
 * written for checking by eye against the paper and the readings listed with
 * each function.
 *
 * Paper: HEP-Frame, arXiv:2211.14346.
 *   - cut pipeline whose cuts each return a boolean (section 3), the last cut
 *     being the kinematic reconstruction that discards events without a
 *     solution (section 4);
 *   - cut reordering driven by filter ratio and measured time, respecting
 *     dependencies, starting from the user's order (section 5.2);
 *   - reconstruction of the two neutrinos from the W (80.4 GeV) and top
 *     (172.5 GeV) mass constraints for every lepton / b-jet pairing, keeping
 *     the most probable solution (section 4);
 *   - pseudo-experiments: energies and momenta varied within a resolution,
 *     keeping the most probable solution (section 4, ttH_sci);
 *   - one-lepton final states: E_T^miss as the neutrino's transverse
 *     momentum, its p_z from the W mass, and the jet assignment that
 *     minimises the chi^2 of Eq. (chi2) with the section 6.2 masses and
 *     widths;
 *   - eta = -ln tan(theta/2) and Delta R = sqrt(Delta eta^2 + Delta phi^2)
 *     (section 6.1 footnote); E_T^miss > 30 GeV, M_ll > 40 GeV, eta regions
 *     (section 6.1); unset variables default to -9999 (section 6.1 example).
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC.
 * Every floating-point operation is IEEE double with no contraction.
 *
 * Parity pins live in tests/test_oracle_*.py.  The choice rule of the
 * reconstruction (which solution is "most probable") has no external
 * reference; that part is "parity unpinned" beyond its closure property.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ types */

#include "orc_events.h"

enum {
    ORC_LEP_N_OS = 0, ORC_JET_N_MIN = 1, ORC_BTAG_N_MIN = 2, ORC_BTAG_N_EQ = 3,
    ORC_MET_MIN = 4, ORC_MLL_MIN = 5, ORC_FWD_JET_VETO = 6, ORC_LEP_ISO = 7,
    ORC_RECO = 8, ORC_MTW_MIN = 9, ORC_USER = 10, ORC_JET_N_RANGE = 11
};

typedef struct {
    int32_t kind;
    int32_t pad;
    double f[8];
    int32_t i[4];
    uint64_t dep_mask;
} orc_cut;

enum { ORC_BTAG_FILL = 0, ORC_ALL_JETS = 1 };

typedef struct {
    double m_t, m_w, lambda_pt;
    double jet_a, jet_c, lep_sigma, met_sigma;
    double lep_pt_min, lep_eta_max, jet_pt_min, jet_eta_max, btag_min;
    uint64_t seed;
    int32_t smear, n_var_uniform, pair_mode, max_cands, want_mbb, pad;
} orc_reco_params;

typedef struct {
    uint8_t *has_sol;
    int32_t *n_sol, *best_v;
    int16_t *best_i, *best_j;
    double *nu;     /* [S][3] */
    double *nubar;  /* [S][3] */
    double *m_t, *m_tbar, *m_wp, *m_wm, *logw, *m_bb;
} orc_reco_out;

typedef struct { double e, x, y, z; } vec4;

#define ORC_NOSOL (-9999.0)
#define ORC_MAX_CANDS 64

/* --------------------------------------------------- counter-based RNG
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplications
 * with the round keys bumped by the Weyl constants between rounds.
 * The paper's own generator is Mersenne Twister (section 5.3), which is
 * sequential; a counter-based generator keyed by (event, variation) is used
 * so that any implementation can reproduce the same draws.            */

void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform in (0,1) from the top 24 bits: u = (floor(x / 2^8) + 1/2) / 2^24. */
static double orc_uniform(uint32_t x)
{
    return ((double)(x >> 8) + 0.5) * (1.0 / 16777216.0);
}

/* Standard normal draw for Gaussian slot `slot` of variation v of global
 * event g.  Slot s lives in Philox block s/4 at lane s%4; lanes (0,1) and
 * (2,3) of a block form Box-Muller pairs (radius from the first, angle from
 * the second; cosine for the first lane, sine for the second). */
double orc_gauss(uint64_t seed, uint64_t g, uint32_t v, uint32_t slot)
{
    uint32_t ctr[4] = {(uint32_t)g, (uint32_t)(g >> 32), v, slot / 4u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t r[4];
    orc_philox4x32_10(ctr, key, r);
    uint32_t lane = slot % 4u;
    uint32_t first = lane & 2u;
    double u1 = orc_uniform(r[first]);
    double u2 = orc_uniform(r[first + 1]);
    double rad = sqrt(-2.0 * log(u1));
    double ang = 2.0 * M_PI * u2;
    return (lane & 1u) ? rad * sin(ang) : rad * cos(ang);
}

/* ------------------------------------------------------------ kinematics */

static vec4 orc_from_polar(double pt, double eta, double phi, double e)
{
    vec4 v;
    v.e = e;
    v.x = pt * cos(phi);
    v.y = pt * sin(phi);
    v.z = pt * sinh(eta);
    return v;
}

static double orc_dot(vec4 a, vec4 b) { return a.e * b.e - a.x * b.x - a.y * b.y - a.z * b.z; }

static vec4 orc_add(vec4 a, vec4 b)
{
    vec4 r = {a.e + b.e, a.x + b.x, a.y + b.y, a.z + b.z};
    return r;
}

static vec4 orc_scale(vec4 a, double s)
{
    vec4 r = {a.e * s, a.x * s, a.y * s, a.z * s};
    return r;
}

static double orc_mass(vec4 a)
{
    double m2 = orc_dot(a, a);
    return m2 > 0.0 ? sqrt(m2) : 0.0;
}

/* Delta phi folded into [-pi, pi]. */
static double orc_dphi(double a, double b)
{
    double d = a - b;
    while (d > M_PI) d -= 2.0 * M_PI;
    while (d < -M_PI) d += 2.0 * M_PI;
    return d;
}

/* ------------------------------------------------------------- selection
 * Object selection reading: a lepton (jet) is selected if pT > pt_min and
 * |eta| < eta_max; a selected jet is b-tagged if btag > btag_min.  Each cut
 * is one boolean predicate of the event (section 3).  Section 6.1 supplies
 * the isolation (Delta R), missing-energy, M_ll and eta-region cuts.      */

static int orc_lep_sel(const orc_events *ev, uint32_t k, double ptmin, double etamax)
{
    return ev->lep_pt[k] > ptmin && fabs(ev->lep_eta[k]) < etamax;
}

static int orc_jet_sel(const orc_events *ev, uint32_t k, double ptmin, double etamax)
{
    return ev->jet_pt[k] > ptmin && fabs(ev->jet_eta[k]) < etamax;
}

static int orc_eval_cut(const orc_events *ev, int64_t e, const orc_cut *c, const orc_user_fn *user)
{
    if (c->kind == ORC_USER) /* a user predicate (section 3: a cut is a boolean function of one event) */
        return user && user[c->i[0]] ? user[c->i[0]](ev, e, c->i[1]) != 0 : 0;
    uint32_t l0 = ev->lep_off[e], l1 = ev->lep_off[e + 1];
    uint32_t j0 = ev->jet_off[e], j1 = ev->jet_off[e + 1];
    switch (c->kind) {
    case ORC_LEP_N_OS: {
        int n = 0;
        double qprod = 1.0;
        for (uint32_t k = l0; k < l1; ++k)
            if (orc_lep_sel(ev, k, c->f[0], c->f[1])) {
                ++n;
                qprod *= ev->lep_q[k];
            }
        if (n != c->i[0]) return 0;
        if (c->i[1] && n == 2 && !(qprod < 0.0)) return 0;
        return 1;
    }
    case ORC_JET_N_MIN: {
        int n = 0;
        for (uint32_t k = j0; k < j1; ++k) n += orc_jet_sel(ev, k, c->f[0], c->f[1]);
        return n >= c->i[0];
    }
    case ORC_BTAG_N_MIN:
    case ORC_BTAG_N_EQ: {
        int n = 0;
        for (uint32_t k = j0; k < j1; ++k)
            n += orc_jet_sel(ev, k, c->f[0], c->f[1]) && ev->jet_btag[k] > c->f[2];
        return c->kind == ORC_BTAG_N_MIN ? n >= c->i[0] : n == c->i[0];
    }
    case ORC_MET_MIN: {
        double met = sqrt(ev->met_x[e] * ev->met_x[e] + ev->met_y[e] * ev->met_y[e]);
        return met > c->f[0];
    }
    case ORC_MLL_MIN: {
        /* invariant mass of the two leading selected leptons */
        vec4 s = {0, 0, 0, 0};
        int n = 0;
        for (uint32_t k = l0; k < l1 && n < 2; ++k)
            if (orc_lep_sel(ev, k, c->f[0], c->f[1])) {
                s = orc_add(s, orc_from_polar(ev->lep_pt[k], ev->lep_eta[k], ev->lep_phi[k], ev->lep_e[k]));
                ++n;
            }
        if (n < 2) return 0;
        double m2 = orc_dot(s, s);
        return m2 > 0.0 && sqrt(m2) > c->f[2];
    }
    case ORC_JET_N_RANGE: {
        /* jets with pT above the threshold in a band of |eta| (section 6.1:
         * Region I |eta| < 2.5, Region II 2.5-2.75, Region III 2.75-3.5),
         * their number within [n_min, n_max] */
        int n = 0;
        for (uint32_t k = j0; k < j1; ++k) {
            double ae = fabs(ev->jet_eta[k]);
            n += ev->jet_pt[k] > c->f[0] && ae >= c->f[1] && ae < c->f[2];
        }
        return n >= c->i[0] && n <= c->i[1];
    }
    case ORC_FWD_JET_VETO: {
        for (uint32_t k = j0; k < j1; ++k) {
            double ae = fabs(ev->jet_eta[k]);
            if (ev->jet_pt[k] > c->f[0] && ae >= c->f[1] && ae < c->f[2]) return 0;
        }
        return 1;
    }
    case ORC_LEP_ISO: {
        /* isolated: no selected jet within Delta R < dr_min of any selected lepton */
        for (uint32_t a = l0; a < l1; ++a) {
            if (!orc_lep_sel(ev, a, c->f[0], c->f[1])) continue;
            for (uint32_t k = j0; k < j1; ++k) {
                if (!orc_jet_sel(ev, k, c->f[2], c->f[3])) continue;
                double deta = ev->lep_eta[a] - ev->jet_eta[k];
                double dphi = orc_dphi(ev->lep_phi[a], ev->jet_phi[k]);
                double dr = sqrt(deta * deta + dphi * dphi);
                if (dr < c->f[4]) return 0;
            }
        }
        return 1;
    }
    case ORC_MTW_MIN: {
        /* W transverse mass of the leading selected lepton and the missing
         * transverse momentum (section 6.1: M_T^W above 50 GeV in the Wt
         * semileptonic bins): M_T^2 = 2 (pT_l E_T^miss - pT_l . MET) */
        for (uint32_t a = l0; a < l1; ++a) {
            if (!orc_lep_sel(ev, a, c->f[0], c->f[1])) continue;
            double pt = ev->lep_pt[a];
            double px = pt * cos(ev->lep_phi[a]), py = pt * sin(ev->lep_phi[a]);
            double mx = ev->met_x[e], my = ev->met_y[e];
            double met = sqrt(mx * mx + my * my);
            double mt2 = 2.0 * (pt * met - (px * mx + py * my));
            return mt2 > c->f[2] * c->f[2];
        }
        return 0;
    }
    default:
        return 1; /* RECO is evaluated by the reconstruction itself */
    }
}

/* Evaluate the cut chain in `order` for every event.  For the cut at
 * position k: reached counts events that survived positions 0..k-1, passed
 * counts those that also survive position k (indexed by cut id, added to
 * the caller's totals).  survive[e] is the AND over all non-RECO cuts.    */
int orc_select_user(const orc_events *ev, const orc_cut *cuts, int n_cuts, const int32_t *order,
                    const orc_user_fn *user, uint8_t *survive, uint64_t *reached, uint64_t *passed)
{
    for (int64_t e = 0; e < ev->n; ++e) {
        int alive = 1;
        for (int k = 0; k < n_cuts && alive; ++k) {
            int c = order[k];
            if (cuts[c].kind == ORC_RECO) continue;
            reached[c] += 1;
            alive = orc_eval_cut(ev, e, &cuts[c], user);
            passed[c] += alive ? 1 : 0;
        }
        survive[e] = (uint8_t)alive;
    }
    return 0;
}

int orc_select(const orc_events *ev, const orc_cut *cuts, int n_cuts, const int32_t *order,
               uint8_t *survive, uint64_t *reached, uint64_t *passed)
{
    return orc_select_user(ev, cuts, n_cuts, order, NULL, survive, reached, passed);
}

/* Survivors in ascending order: idx[s] = map ? map[e] : index_base + e. */
int64_t orc_compact(const uint8_t *mask, int64_t n, int64_t index_base, const int32_t *map, int32_t *idx)
{
    int64_t s = 0;
    for (int64_t e = 0; e < n; ++e)
        if (mask[e]) idx[s++] = map ? map[e] : (int32_t)(index_base + e);
    return s;
}

/* ----------------------------------------------------------- reordering
 * Section 5.2: cuts that filter out more events go earlier and heavier cuts
 * later, respecting dependencies, starting from the user's order.
 * Reading: pass rate p = passed/reached (1 if never reached), per-event cost
 * c = cost/reached (0 if never reached), rank r = c / max(1 - p, 1e-9).
 * Repeatedly place, among cuts whose dependencies are already placed, the one
 * with the smallest rank; ties go to the lower cut id.                    */
int orc_reorder(const uint64_t *reached, const uint64_t *passed, const uint64_t *cost,
                const uint64_t *dep_mask, int n, int32_t *order)
{
    uint64_t placed = 0;
    for (int pos = 0; pos < n; ++pos) {
        int best = -1;
        double best_r = 0.0;
        for (int c = 0; c < n; ++c) {
            if (placed & (1ull << c)) continue;
            if ((dep_mask[c] & ~placed) != 0) continue;
            double p = reached[c] ? (double)passed[c] / (double)reached[c] : 1.0;
            double cc = reached[c] ? (double)cost[c] / (double)reached[c] : 0.0;
            double d = 1.0 - p;
            double r = cc / (d > 1e-9 ? d : 1e-9);
            if (best < 0 || r < best_r) {
                best = c;
                best_r = r;
            }
        }
        if (best < 0) return -1; /* cyclic dependencies */
        order[pos] = best;
        placed |= 1ull << best;
    }
    return 0;
}

/* ------------------------------------------------ polynomial real roots
 * Real roots by critical-point isolation: the real roots of p' split the
 * line into intervals on which p is monotone; each interval whose end values
 * differ in sign holds exactly one root, found by bisection down to two ulp.
 * The recursion bottoms out at the quadratic p'' of a quartic, solved in
 * closed form.  Only sign-changing roots are reported (a root of even
 * multiplicity is not).  The outer intervals end at the Cauchy bound.     */

static double orc_horner(const double *c, int n, double x)
{
    double r = c[n];
    for (int i = n - 1; i >= 0; --i) r = r * x + c[i];
    return r;
}

static double orc_ulp(double x)
{
    x = fabs(x);
    return nextafter(x, INFINITY) - x;
}

static double orc_bisect(const double *c, int n, double lo, double hi)
{
    double flo = orc_horner(c, n, lo);
    for (int it = 0; it < 4000; ++it) {
        double w = fabs(lo) > fabs(hi) ? fabs(lo) : fabs(hi);
        if (hi - lo <= 2.0 * orc_ulp(w)) break;
        double mid = lo + 0.5 * (hi - lo);
        if (!(mid > lo && mid < hi)) break;
        double fm = orc_horner(c, n, mid);
        if (fm == 0.0) return mid;
        if ((fm < 0.0) == (flo < 0.0)) {
            lo = mid;
            flo = fm;
        } else {
            hi = mid;
        }
    }
    return lo + 0.5 * (hi - lo);
}

/* c[0..n] with c[n] != 0; roots written ascending; returns their number. */
static int orc_roots_rec(const double *c, int n, double *out)
{
    if (n <= 0) return 0;
    if (n == 1) {
        out[0] = -c[0] / c[1];
        return 1;
    }
    if (n == 2) {
        double disc = c[1] * c[1] - 4.0 * c[2] * c[0];
        if (!(disc > 0.0)) return 0;
        double s = sqrt(disc);
        double t = -0.5 * (c[1] + (c[1] >= 0.0 ? s : -s));
        double r1 = t / c[2];
        double r2 = c[0] / t;
        out[0] = r1 < r2 ? r1 : r2;
        out[1] = r1 < r2 ? r2 : r1;
        return 2;
    }
    double d[8];
    for (int i = 1; i <= n; ++i) d[i - 1] = (double)i * c[i];
    double crit[8];
    int nc = orc_roots_rec(d, n - 1, crit);
    double bound = 0.0;
    for (int i = 0; i < n; ++i) {
        double r = fabs(c[i] / c[n]);
        if (r > bound) bound = r;
    }
    bound += 1.0;
    double pts[10];
    int m = 0;
    pts[m++] = -bound;
    for (int k = 0; k < nc; ++k) pts[m++] = crit[k];
    pts[m++] = bound;
    int nr = 0;
    for (int k = 0; k + 1 < m; ++k) {
        double lo = pts[k], hi = pts[k + 1];
        if (!(hi > lo)) continue;
        double flo = orc_horner(c, n, lo), fhi = orc_horner(c, n, hi);
        if ((flo < 0.0 && fhi > 0.0) || (flo > 0.0 && fhi < 0.0)) out[nr++] = orc_bisect(c, n, lo, hi);
    }
    return nr;
}

/* Real roots of c[0] + c[1] t + ... + c[4] t^4.  Reading: coefficients are
 * normalised by max |c_i|, and trailing coefficients of magnitude <= 1e-14
 * are dropped (degree reduction).  Returns the count; roots ascending.   */
int orc_real_roots(const double c_in[5], double roots[4])
{
    double mx = 0.0;
    for (int i = 0; i < 5; ++i)
        if (fabs(c_in[i]) > mx) mx = fabs(c_in[i]);
    if (!(mx > 0.0) || !isfinite(mx)) return 0;
    double c[5];
    for (int i = 0; i < 5; ++i) c[i] = c_in[i] / mx;
    int n = 4;
    while (n > 0 && fabs(c[n]) <= 1e-14) --n;
    return orc_roots_rec(c, n, roots);
}

/* --------------------------------------------- two-neutrino reconstruction
 * Unknowns: neutrino nu = (E, x, y, z) from t -> b l+ nu and antineutrino
 * nubar from tbar -> bbar l- nubar.  Constraints (section 4): (l+nu)^2 = mW^2,
 * (b+l+nu)^2 = mt^2 and the same for the antitop, massless neutrinos, and
 * transverse momentum balance nu_T + nubar_T = MET.
 *
 * With m_nu = 0, (l+nu)^2 = mW^2 gives l.nu = kl = (mW^2 - ml^2)/2 and
 * (b+l+nu)^2 = mt^2 gives b.nu = kb = (mt^2 - mW^2 - mb^2 - 2 b.l)/2.  These
 * two equations are linear in (E, z) for given (x, y):
 *     El E - lz z = kl + lx x + ly y,   Eb E - bz z = kb + bx x + by y,
 * solved by Cramer's rule (determinant D = lz Eb - El bz).  The mass shell
 * E^2 - x^2 - y^2 - z^2 = 0 then is a conic in (x, y).  The antineutrino gives
 * a conic in (xb, yb) = (METx - x, METy - y).  Eliminating y from the two
 * conics (resultant) leaves a quartic in x.                              */

typedef struct {
    /* E = ex x + ey y + e0 ; z = zx x + zy y + z0 */
    double ex, ey, e0, zx, zy, z0;
    int ok;
} orc_linmap;

static orc_linmap orc_linear_map(vec4 l, vec4 b, double mt, double mw)
{
    orc_linmap m;
    double ml2 = orc_dot(l, l), mb2 = orc_dot(b, b);
    double kl = 0.5 * (mw * mw - ml2);
    double kb = 0.5 * (mt * mt - mw * mw - mb2 - 2.0 * orc_dot(b, l));
    /* system  [El -lz; Eb -bz] [E; z] = [r1; r2] */
    double det = l.z * b.e - l.e * b.z; /* = El*(-bz) - (-lz)*Eb */
    /* Reading: the system is treated as degenerate when |det| <= 1e-5 El Eb
     * (for massless l and b: their direction cosines along the beam agree to
     * 1e-5).  The map's coefficients grow as 1/det and the rounding of the
     * mass shell faster still; below this bound FP64 no longer resolves the
     * constraints to the acceptance bound used below. */
    m.ok = fabs(det) > 1e-5 * l.e * b.e;
    if (!m.ok) return m;
    /* Cramer: E = (r1*(-bz) - (-lz)*r2)/det, z = (El*r2 - Eb*r1)/det, applied to
     * each of the three right-hand-side components (x coeff, y coeff, constant). */
    double r1[3] = {l.x, l.y, kl};
    double r2[3] = {b.x, b.y, kb};
    double ec[3], zc[3];
    for (int k = 0; k < 3; ++k) {
        ec[k] = (r1[k] * (-b.z) - (-l.z) * r2[k]) / det;
        zc[k] = (l.e * r2[k] - b.e * r1[k]) / det;
    }
    m.ex = ec[0]; m.ey = ec[1]; m.e0 = ec[2];
    m.zx = zc[0]; m.zy = zc[1]; m.z0 = zc[2];
    return m;
}

/* Bivariate quadratic q(x,y) = xx x^2 + xy x y + yy y^2 + x_ x + y_ y + c. */
typedef struct { double xx, xy, yy, x_, y_, c; } orc_conic;

/* E^2 - x^2 - y^2 - z^2 with E and z affine in (x, y). */
static orc_conic orc_shell_conic(orc_linmap m)
{
    orc_conic q;
    q.xx = m.ex * m.ex - 1.0 - m.zx * m.zx;
    q.xy = 2.0 * (m.ex * m.ey - m.zx * m.zy);
    q.yy = m.ey * m.ey - 1.0 - m.zy * m.zy;
    q.x_ = 2.0 * (m.ex * m.e0 - m.zx * m.z0);
    q.y_ = 2.0 * (m.ey * m.e0 - m.zy * m.z0);
    q.c = m.e0 * m.e0 - m.z0 * m.z0;
    return q;
}

/* q(mx - x, my - y) expanded as a conic in (x, y). */
static orc_conic orc_reflect_conic(orc_conic q, double mx, double my)
{
    orc_conic r;
    r.xx = q.xx;
    r.xy = q.xy;
    r.yy = q.yy;
    r.x_ = -2.0 * q.xx * mx - q.xy * my - q.x_;
    r.y_ = -q.xy * mx - 2.0 * q.yy * my - q.y_;
    r.c = q.xx * mx * mx + q.xy * mx * my + q.yy * my * my + q.x_ * mx + q.y_ * my + q.c;
    return r;
}

static double orc_conic_eval(orc_conic q, double x, double y)
{
    return q.xx * x * x + q.xy * x * y + q.yy * y * y + q.x_ * x + q.y_ * y + q.c;
}

/* |q(x,y)| relative to the sum of the magnitudes of its terms */
static double orc_conic_rel(orc_conic q, double x, double y, double val)
{
    double s = fabs(q.xx * x * x) + fabs(q.xy * x * y) + fabs(q.yy * y * y) + fabs(q.x_ * x) +
               fabs(q.y_ * y) + fabs(q.c);
    return s > 0.0 ? fabs(val) / s : 0.0;
}

/* small dense polynomials in x, coefficient i multiplies x^i */
typedef struct { double c[5]; int n; } orc_poly; /* degree n */

static orc_poly orc_pmul(orc_poly a, orc_poly b)
{
    orc_poly r;
    memset(&r, 0, sizeof r);
    r.n = a.n + b.n;
    for (int i = 0; i <= a.n; ++i)
        for (int j = 0; j <= b.n; ++j) r.c[i + j] += a.c[i] * b.c[j];
    return r;
}

static orc_poly orc_psub(orc_poly a, orc_poly b)
{
    orc_poly r;
    memset(&r, 0, sizeof r);
    r.n = a.n > b.n ? a.n : b.n;
    for (int i = 0; i <= r.n; ++i) r.c[i] = (i <= a.n ? a.c[i] : 0.0) - (i <= b.n ? b.c[i] : 0.0);
    return r;
}

static double orc_peval(orc_poly p, double x) { return orc_horner(p.c, p.n, x); }

/* Scale of the variable in which the quartic is normalised and solved:
 * x = ORC_XSCALE * t (reading; keeps the degree test scale-free in GeV). */
#define ORC_XSCALE 100.0

/* Real roots of a y^2 + b y + c (linear if a == 0); returns count (0..2). */
static int orc_quad_roots(double a, double b, double c, double *out)
{
    if (a == 0.0) {
        if (b == 0.0) return 0;
        out[0] = -c / b;
        return 1;
    }
    double disc = b * b - 4.0 * a * c;
    if (disc < 0.0) return 0;
    double s = sqrt(disc);
    double t = -0.5 * (b + (b >= 0.0 ? s : -s));
    if (t == 0.0) {
        out[0] = 0.0;
        return 1;
    }
    out[0] = t / a;
    out[1] = c / t;
    return 2;
}

typedef struct {
    double x, y, z, e;      /* neutrino */
    double xb, yb, zb, eb;  /* antineutrino */
} orc_solution;

/* All accepted solutions for one pairing, ascending in x; returns count. */
int orc_solve_pairing_v(vec4 lp, vec4 b, vec4 lm, vec4 bb, double metx, double mety,
                        double mt, double mw, orc_solution *sol)
{
    orc_linmap m1 = orc_linear_map(lp, b, mt, mw);
    orc_linmap m2 = orc_linear_map(lm, bb, mt, mw);
    if (!m1.ok || !m2.ok) return 0;
    orc_conic c1 = orc_shell_conic(m1);
    orc_conic c2 = orc_reflect_conic(orc_shell_conic(m2), metx, mety);
    /* P(y) = a y^2 + b(x) y + c(x),  Q(y) = d y^2 + e(x) y + f(x) */
    orc_poly pa = {{c1.yy}, 0}, pb = {{c1.y_, c1.xy}, 1}, pc = {{c1.c, c1.x_, c1.xx}, 2};
    orc_poly qd = {{c2.yy}, 0}, qe = {{c2.y_, c2.xy}, 1}, qf = {{c2.c, c2.x_, c2.xx}, 2};
    /* Res_y(P, Q) = (a f - c d)^2 - (a e - b d)(b f - c e) */
    orc_poly g = orc_psub(orc_pmul(pa, qf), orc_pmul(pc, qd));
    orc_poly h = orc_psub(orc_pmul(pa, qe), orc_pmul(pb, qd));
    orc_poly k = orc_psub(orc_pmul(pb, qf), orc_pmul(pc, qe));
    orc_poly res = orc_psub(orc_pmul(g, g), orc_pmul(h, k));
    double ct[5];
    double sc = 1.0;
    for (int i = 0; i < 5; ++i) {
        ct[i] = (i <= res.n ? res.c[i] : 0.0) * sc; /* coefficients in t = x / XSCALE */
        sc *= ORC_XSCALE;
    }
    double troots[4];
    int nr = orc_real_roots(ct, troots);
    int ns = 0;
    for (int r = 0; r < nr; ++r) {
        double x = ORC_XSCALE * troots[r];
        double a = pa.c[0], d = qd.c[0];
        double bx = orc_peval(pb, x), cx = orc_peval(pc, x);
        double ex = orc_peval(qe, x), fx = orc_peval(qf, x);
        /* y is the common root of P(y) = a y^2 + bx y + cx and Q(y) = d y^2 + ex y + fx.
         * Candidates: the elimination a Q - d P = (a ex - bx d) y + (a fx - cx d) = 0, and
         * the real roots of P and of Q.  Keep the candidate with the smallest sum of the
         * two relative residuals (reading: the elimination alone loses all precision
         * when two intersection points share nearly the same x). */
        double cand[5];
        int ncand = 0;
        double den = bx * d - a * ex;
        if (den != 0.0) cand[ncand++] = (a * fx - cx * d) / den;
        ncand += orc_quad_roots(a, bx, cx, cand + ncand);
        ncand += orc_quad_roots(d, ex, fx, cand + ncand);
        if (ncand == 0) continue;
        double y = cand[0], best_res = INFINITY;
        for (int q = 0; q < ncand; ++q) {
            double yy = cand[q];
            double rp = fabs(a * yy * yy + bx * yy + cx) / (fabs(a) * yy * yy + fabs(bx * yy) + fabs(cx));
            double rq = fabs(d * yy * yy + ex * yy + fx) / (fabs(d) * yy * yy + fabs(ex * yy) + fabs(fx));
            double res = rp + rq;
            if (res < best_res) {
                best_res = res;
                y = yy;
            }
        }
        /* Polish (x, y) by Newton's method on the two conics themselves, whose
         * coefficients carry far less cancellation than the expanded quartic; a
         * step is kept only while it lowers the larger relative residual. */
        for (int it = 0; it < 4; ++it) {
            double f1 = orc_conic_eval(c1, x, y), f2 = orc_conic_eval(c2, x, y);
            double r0 = orc_conic_rel(c1, x, y, f1);
            double r1 = orc_conic_rel(c2, x, y, f2);
            double rmax = r0 > r1 ? r0 : r1;
            if (rmax == 0.0) break;
            double a11 = 2.0 * c1.xx * x + c1.xy * y + c1.x_, a12 = c1.xy * x + 2.0 * c1.yy * y + c1.y_;
            double a21 = 2.0 * c2.xx * x + c2.xy * y + c2.x_, a22 = c2.xy * x + 2.0 * c2.yy * y + c2.y_;
            double det = a11 * a22 - a12 * a21;
            if (det == 0.0) break;
            double dx = (-f1 * a22 + f2 * a12) / det;
            double dy = (-a11 * f2 + a21 * f1) / det;
            double xn = x + dx, yn = y + dy;
            double g1 = orc_conic_eval(c1, xn, yn), g2 = orc_conic_eval(c2, xn, yn);
            double s0 = orc_conic_rel(c1, xn, yn, g1), s1 = orc_conic_rel(c2, xn, yn, g2);
            if (!((s0 > s1 ? s0 : s1) < rmax)) break;
            x = xn;
            y = yn;
        }
        /* A root of the eliminant only says the two conics share a root in y; the
         * point is a solution of the mass constraints (section 4) only if both
         * conics vanish there.  The W and top constraints hold by construction
         * of the linear maps, and each conic's value is that neutrino's squared
         * mass E^2 - p^2 in GeV^2, so (l + nu)^2 - mW^2 and (b + l + nu)^2 - mt^2
         * both equal it.  Reading: accept when both squared masses are within
         * 2e-6 mW^2 of zero after the polish (every mass constraint then holds to
         * 1e-6 relative), which also rejects near-tangent artefacts. */
        {
            double tol = 2e-6 * mw * mw;
            if (!(fabs(orc_conic_eval(c1, x, y)) <= tol && fabs(orc_conic_eval(c2, x, y)) <= tol)) continue;
        }
        double xb = metx - x, yb = mety - y;
        double en = m1.ex * x + m1.ey * y + m1.e0;
        double zn = m1.zx * x + m1.zy * y + m1.z0;
        double eb = m2.ex * xb + m2.ey * yb + m2.e0;
        double zb = m2.zx * xb + m2.zy * yb + m2.z0;
        /* squaring introduced negative-energy branches: reject them */
        if (en < 0.0 || eb < 0.0) continue;
        orc_solution s = {x, y, zn, en, xb, yb, zb, eb};
        sol[ns++] = s;
    }
    return ns;
}

/* ctypes-friendly form: vectors as (E, px, py, pz); out[k*8 + ...] holds
 * x, y, z, E of nu then x, y, z, E of nubar. */
int orc_solve_pairing(const double lp[4], const double b[4], const double lm[4], const double bb[4],
                      double metx, double mety, double mt, double mw, double *out)
{
    vec4 a = {lp[0], lp[1], lp[2], lp[3]}, bq = {b[0], b[1], b[2], b[3]};
    vec4 c = {lm[0], lm[1], lm[2], lm[3]}, d = {bb[0], bb[1], bb[2], bb[3]};
    orc_solution s[4];
    int n = orc_solve_pairing_v(a, bq, c, d, metx, mety, mt, mw, s);
    for (int k = 0; k < n; ++k) {
        double *o = out + 8 * k;
        o[0] = s[k].x; o[1] = s[k].y; o[2] = s[k].z; o[3] = s[k].e;
        o[4] = s[k].xb; o[5] = s[k].yb; o[6] = s[k].zb; o[7] = s[k].eb;
    }
    return n;
}

/* Quartic coefficients (in x, GeV units) for one pairing, for tests. */
int orc_pairing_quartic(const double lp[4], const double b[4], const double lm[4], const double bb[4],
                        double metx, double mety, double mt, double mw, double out[5])
{
    vec4 a = {lp[0], lp[1], lp[2], lp[3]}, bq = {b[0], b[1], b[2], b[3]};
    vec4 c = {lm[0], lm[1], lm[2], lm[3]}, d = {bb[0], bb[1], bb[2], bb[3]};
    orc_linmap m1 = orc_linear_map(a, bq, mt, mw), m2 = orc_linear_map(c, d, mt, mw);
    if (!m1.ok || !m2.ok) return 0;
    orc_conic c1 = orc_shell_conic(m1);
    orc_conic c2 = orc_reflect_conic(orc_shell_conic(m2), metx, mety);
    orc_poly pa = {{c1.yy}, 0}, pb = {{c1.y_, c1.xy}, 1}, pc = {{c1.c, c1.x_, c1.xx}, 2};
    orc_poly qd = {{c2.yy}, 0}, qe = {{c2.y_, c2.xy}, 1}, qf = {{c2.c, c2.x_, c2.xx}, 2};
    orc_poly g = orc_psub(orc_pmul(pa, qf), orc_pmul(pc, qd));
    orc_poly h = orc_psub(orc_pmul(pa, qe), orc_pmul(pb, qd));
    orc_poly k = orc_psub(orc_pmul(pb, qf), orc_pmul(pc, qe));
    orc_poly res = orc_psub(orc_pmul(g, g), orc_pmul(h, k));
    for (int i = 0; i < 5; ++i) out[i] = i <= res.n ? res.c[i] : 0.0;
    return 1;
}

/* ------------------------------------------------- per-event reconstruction */

typedef struct {
    int ok;
    int leps;                  /* two selected opposite-sign leptons */
    vec4 lp, lm;
    int nc;
    int cand[ORC_MAX_CANDS];   /* jet index within the event, candidate order */
    vec4 cv[ORC_MAX_CANDS];
    double sigma[ORC_MAX_CANDS];
} orc_staged;

/* Leptons: the two selected ones, l+ the positive.  b candidates (reading):
 * BTAG_FILL takes the b-tagged selected jets in input (pT) order, capped at
 * max_cands, filled up to two with the leading untagged selected jets;
 * ALL_JETS takes every selected jet up to max_cands. */
static orc_staged orc_stage(const orc_events *ev, int64_t e, const orc_reco_params *p)
{
    orc_staged s;
    memset(&s, 0, sizeof s);
    uint32_t l0 = ev->lep_off[e], l1 = ev->lep_off[e + 1];
    uint32_t j0 = ev->jet_off[e], j1 = ev->jet_off[e + 1];
    int nl = 0;
    uint32_t lk[2] = {0, 0};
    for (uint32_t k = l0; k < l1; ++k)
        if (orc_lep_sel(ev, k, p->lep_pt_min, p->lep_eta_max)) {
            if (nl < 2) lk[nl] = k;
            ++nl;
        }
    if (nl != 2 || !(ev->lep_q[lk[0]] * ev->lep_q[lk[1]] < 0.0)) return s;
    s.leps = 1;
    uint32_t kp = ev->lep_q[lk[0]] > 0.0 ? lk[0] : lk[1];
    uint32_t km = ev->lep_q[lk[0]] > 0.0 ? lk[1] : lk[0];
    s.lp = orc_from_polar(ev->lep_pt[kp], ev->lep_eta[kp], ev->lep_phi[kp], ev->lep_e[kp]);
    s.lm = orc_from_polar(ev->lep_pt[km], ev->lep_eta[km], ev->lep_phi[km], ev->lep_e[km]);
    int cap = p->max_cands < ORC_MAX_CANDS ? p->max_cands : ORC_MAX_CANDS;
    int nc = 0;
    if (p->pair_mode == ORC_ALL_JETS) {
        for (uint32_t k = j0; k < j1 && nc < cap; ++k)
            if (orc_jet_sel(ev, k, p->jet_pt_min, p->jet_eta_max)) s.cand[nc++] = (int)(k - j0);
    } else {
        for (uint32_t k = j0; k < j1 && nc < cap; ++k)
            if (orc_jet_sel(ev, k, p->jet_pt_min, p->jet_eta_max) && ev->jet_btag[k] > p->btag_min)
                s.cand[nc++] = (int)(k - j0);
        for (uint32_t k = j0; k < j1 && nc < 2; ++k)
            if (orc_jet_sel(ev, k, p->jet_pt_min, p->jet_eta_max) && !(ev->jet_btag[k] > p->btag_min))
                s.cand[nc++] = (int)(k - j0);
    }
    s.nc = nc;
    for (int c = 0; c < nc; ++c) {
        uint32_t k = j0 + (uint32_t)s.cand[c];
        s.cv[c] = orc_from_polar(ev->jet_pt[k], ev->jet_eta[k], ev->jet_phi[k], ev->jet_e[k]);
        /* jet resolution: sigma_E/E = a/sqrt(E) (+) c, at the nominal energy */
        s.sigma[c] = sqrt(p->jet_a * p->jet_a / ev->jet_e[k] + p->jet_c * p->jet_c);
    }
    s.ok = nc >= 2;
    return s;
}

static double orc_smear_factor(double sigma, double z)
{
    double s = 1.0 + sigma * z;
    return s > 0.01 ? s : 0.01;
}

/* One resolution variation of a staged event (reading of section 4's
 * pseudo-experiments): Gaussian draws for l+ (slot 0), l- (1), MET x (2),
 * MET y (3) and jet k of the event in input order (4 + k); every 4-vector
 * component scaled by max(1 + sigma z, 0.01); MET shifted by met_sigma z.
 * With smear = 0 every draw is zero. */
typedef struct {
    double z_lp, z_lm, z_mx, z_my;
    double zj[ORC_MAX_CANDS];
    vec4 lp, lm;
    vec4 cv[ORC_MAX_CANDS];
    double mx, my;
} orc_variation;

static void orc_vary(const orc_staged *st, const orc_events *ev, int64_t e, uint64_t g, int v,
                     const orc_reco_params *p, orc_variation *o)
{
    memset(o, 0, sizeof *o);
    if (p->smear) {
        o->z_lp = orc_gauss(p->seed, g, (uint32_t)v, 0);
        o->z_lm = orc_gauss(p->seed, g, (uint32_t)v, 1);
        o->z_mx = orc_gauss(p->seed, g, (uint32_t)v, 2);
        o->z_my = orc_gauss(p->seed, g, (uint32_t)v, 3);
        for (int c = 0; c < st->nc; ++c)
            o->zj[c] = orc_gauss(p->seed, g, (uint32_t)v, 4u + (uint32_t)st->cand[c]);
    }
    o->lp = orc_scale(st->lp, orc_smear_factor(p->lep_sigma, o->z_lp));
    o->lm = orc_scale(st->lm, orc_smear_factor(p->lep_sigma, o->z_lm));
    o->mx = ev->met_x[e] + p->met_sigma * o->z_mx;
    o->my = ev->met_y[e] + p->met_sigma * o->z_my;
    for (int c = 0; c < st->nc; ++c) o->cv[c] = orc_scale(st->cv[c], orc_smear_factor(st->sigma[c], o->zj[c]));
}

/* Inspection of one (event, variation) for the tests: the staged candidates
 * (jet indices within the event) and the varied objects.  Returns -1 when
 * the event does not have two selected opposite-sign leptons, else the
 * number of candidates (which may be below two).  vecs: (E, px, py, pz) of
 * l+, l-, then each candidate; met: shifted (x, y); z: the draws of l+, l-,
 * MET x, MET y, then each candidate.                                      */
int orc_stage_vary(const orc_events *ev, int64_t e, int v, const orc_reco_params *p, int32_t *cand,
                   double *vecs, double *met, double *z)
{
    orc_staged st = orc_stage(ev, e, p);
    if (!st.leps) return -1;
    orc_variation o;
    orc_vary(&st, ev, e, (uint64_t)(ev->index_base + e), v, p, &o);
    const vec4 *all[2 + ORC_MAX_CANDS];
    all[0] = &o.lp;
    all[1] = &o.lm;
    for (int c = 0; c < st.nc; ++c) all[2 + c] = &o.cv[c];
    for (int k = 0; k < 2 + st.nc; ++k) {
        vecs[4 * k + 0] = all[k]->e; vecs[4 * k + 1] = all[k]->x;
        vecs[4 * k + 2] = all[k]->y; vecs[4 * k + 3] = all[k]->z;
    }
    for (int c = 0; c < st.nc; ++c) cand[c] = st.cand[c];
    met[0] = o.mx;
    met[1] = o.my;
    z[0] = o.z_lp; z[1] = o.z_lm; z[2] = o.z_mx; z[3] = o.z_my;
    for (int c = 0; c < st.nc; ++c) z[4 + c] = o.zj[c];
    return st.nc;
}

/* Reconstruct the compacted events idx[0..S) (global ids).  For each event,
 * variation v and pairing (i, j) (candidate i with l+, candidate j with l-,
 * i != j, pairing index p = i*nc + j), every accepted solution is scored by
 *   log w = -1/2 sum z_k^2  -  (pT(t) + pT(tbar)) / lambda
 * over the Gaussian draws z of l+, l-, the two candidates and the two MET
 * components (reading of the paper's per-permutation probability), and the
 * maximum is kept; ties go to the smallest (v, p, x).  Returns the number of
 * events with at least one solution.                                      */
int64_t orc_ttbar_reco(const orc_events *ev, const int32_t *idx, int64_t S, const orc_reco_params *p,
                       const orc_reco_out *out, int n_threads)
{
    int64_t npass = 0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : npass)
#endif
    for (int64_t s = 0; s < S; ++s) {
        int64_t g = idx[s];
        int64_t e = g - ev->index_base;
        orc_staged st = orc_stage(ev, e, p);
        int V = ev->n_var ? ev->n_var[e] : p->n_var_uniform;
        int have = 0, nsol = 0;
        double best_w = 0.0, best_x = 0.0;
        int best_v = -1, best_p = -1, best_i = -1, best_j = -1;
        orc_solution best_s;
        vec4 best_lp = {0, 0, 0, 0}, best_lm = best_lp, best_b = best_lp, best_bb = best_lp;
        memset(&best_s, 0, sizeof best_s);
        if (st.ok) {
            for (int v = 0; v < V; ++v) {
                orc_variation o;
                orc_vary(&st, ev, e, (uint64_t)g, v, p, &o);
                const double z_lp = o.z_lp, z_lm = o.z_lm, z_mx = o.z_mx, z_my = o.z_my;
                const double *zj = o.zj;
                const vec4 lp = o.lp, lm = o.lm;
                const double mx = o.mx, my = o.my;
                for (int i = 0; i < st.nc; ++i) {
                    const vec4 b = o.cv[i];
                    for (int j = 0; j < st.nc; ++j) {
                        if (j == i) continue;
                        const vec4 bb = o.cv[j];
                        orc_solution sol[4];
                        int ns = orc_solve_pairing_v(lp, b, lm, bb, mx, my, p->m_t, p->m_w, sol);
                        nsol += ns;
                        int pidx = i * st.nc + j;
                        for (int r = 0; r < ns; ++r) {
                            double ptt = hypot(b.x + lp.x + sol[r].x, b.y + lp.y + sol[r].y);
                            double pttb = hypot(bb.x + lm.x + sol[r].xb, bb.y + lm.y + sol[r].yb);
                            double zz = z_lp * z_lp + z_lm * z_lm + zj[i] * zj[i] + zj[j] * zj[j] +
                                        z_mx * z_mx + z_my * z_my;
                            double w = -0.5 * zz - (ptt + pttb) / p->lambda_pt;
                            int better = !have || w > best_w ||
                                         (w == best_w && (v < best_v || (v == best_v && (pidx < best_p ||
                                          (pidx == best_p && sol[r].x < best_x)))));
                            if (better) {
                                have = 1;
                                best_w = w; best_v = v; best_p = pidx; best_x = sol[r].x;
                                best_i = i; best_j = j; best_s = sol[r];
                                best_lp = lp; best_lm = lm; best_b = b; best_bb = bb;
                            }
                        }
                    }
                }
            }
        }
        out->n_sol[s] = nsol;
        out->has_sol[s] = (uint8_t)have;
        if (!have) {
            out->best_v[s] = -1;
            out->best_i[s] = -1;
            out->best_j[s] = -1;
            for (int k = 0; k < 3; ++k) out->nu[3 * s + k] = out->nubar[3 * s + k] = ORC_NOSOL;
            out->m_t[s] = out->m_tbar[s] = out->m_wp[s] = out->m_wm[s] = ORC_NOSOL;
            out->logw[s] = ORC_NOSOL;
            if (out->m_bb) out->m_bb[s] = ORC_NOSOL;
            continue;
        }
        ++npass;
        vec4 nu = {best_s.e, best_s.x, best_s.y, best_s.z};
        vec4 nub = {best_s.eb, best_s.xb, best_s.yb, best_s.zb};
        out->best_v[s] = best_v;
        out->best_i[s] = (int16_t)st.cand[best_i];
        out->best_j[s] = (int16_t)st.cand[best_j];
        out->nu[3 * s + 0] = nu.x; out->nu[3 * s + 1] = nu.y; out->nu[3 * s + 2] = nu.z;
        out->nubar[3 * s + 0] = nub.x; out->nubar[3 * s + 1] = nub.y; out->nubar[3 * s + 2] = nub.z;
        out->m_wp[s] = orc_mass(orc_add(best_lp, nu));
        out->m_wm[s] = orc_mass(orc_add(best_lm, nub));
        out->m_t[s] = orc_mass(orc_add(best_b, orc_add(best_lp, nu)));
        out->m_tbar[s] = orc_mass(orc_add(best_bb, orc_add(best_lm, nub)));
        out->logw[s] = best_w;
        if (out->m_bb) {
            /* H -> b bbar candidate from the remaining jets (section 4): the two
             * leading remaining b-tagged selected jets; with only one, pair it
             * with the leading remaining untagged selected jet (reading). */
            double mbb = ORC_NOSOL;
            if (p->want_mbb) {
                uint32_t j0 = ev->jet_off[e], j1 = ev->jet_off[e + 1];
                int bi = st.cand[best_i], bj = st.cand[best_j];
                int got = 0;
                uint32_t pick[2] = {0, 0};
                for (uint32_t k = j0; k < j1 && got < 2; ++k) {
                    int loc = (int)(k - j0);
                    if (loc == bi || loc == bj) continue;
                    if (orc_jet_sel(ev, k, p->jet_pt_min, p->jet_eta_max) && ev->jet_btag[k] > p->btag_min)
                        pick[got++] = k;
                }
                if (got == 1) {
                    for (uint32_t k = j0; k < j1; ++k) {
                        int loc = (int)(k - j0);
                        if (loc == bi || loc == bj) continue;
                        if (orc_jet_sel(ev, k, p->jet_pt_min, p->jet_eta_max) &&
                            !(ev->jet_btag[k] > p->btag_min)) {
                            pick[got++] = k;
                            break;
                        }
                    }
                }
                if (got == 2) {
                    vec4 a = orc_from_polar(ev->jet_pt[pick[0]], ev->jet_eta[pick[0]], ev->jet_phi[pick[0]],
                                            ev->jet_e[pick[0]]);
                    vec4 b = orc_from_polar(ev->jet_pt[pick[1]], ev->jet_eta[pick[1]], ev->jet_phi[pick[1]],
                                            ev->jet_e[pick[1]]);
                    mbb = orc_mass(orc_add(a, b));
                }
            }
            out->m_bb[s] = mbb;
        }
    }
    return npass;
}

/* ----------------------------------------- single-neutrino reconstruction
 * Section 6.2, Eq. (chi2).  One-lepton final states: the missing transverse
 * momentum is the neutrino's transverse momentum and only the neutrino's
 * p_z is unknown; it follows from the W mass.  Among every assignment of the
 * selected jets to the expected top quarks and W bosons, the one with the
 * smallest
 *   chi^2 = sum_k (m_top_k - m_t)^2 / sigma_t^2 + sum_m (m_W_m - m_W)^2 / sigma_W^2
 * is kept.  Topologies (the k and m counts of Eq. (chi2)):
 *   TCHAN  (t-channel single top): one top (j l nu), one W (l nu);
 *   WT     (Wt, semileptonic):     one top (j l nu), two W: (l nu) and the
 *                                  two-jet W (p q) (reading: the hadronic W's
 *                                  mass is that of two further jets);
 *   TTSEMI (semileptonic ttbar):   two tops (j l nu) and (h p q), two W:
 *                                  (l nu) and (p q).
 * Jets j, h, p, q are distinct; p < q.                                     */

enum { ORC_TOPO_TCHAN = 0, ORC_TOPO_WT = 1, ORC_TOPO_TTSEMI = 2 };

typedef struct {
    double m_t, m_w, sigma_t, sigma_w;
    double lep_pt_min, lep_eta_max, jet_pt_min, jet_eta_max;
    int32_t topology, max_cands;
} orc_semilep_params;

typedef struct {
    uint8_t *has_sol;
    int8_t *root;                       /* 0: minus sign, 1: plus sign, 2: real part */
    int16_t *best_j, *best_h, *best_p, *best_q;
    double *nu;                         /* [S][3] */
    double *m_tl, *m_wl, *m_th, *m_wh, *chi2;
} orc_semilep_out;

/* Neutrino p_z from (l + nu)^2 = m_W^2 with nu = (|nu|, metx, mety, p_z)
 * massless.  Writing mu = (m_W^2 - m_l^2)/2 + px_l metx + py_l mety, the
 * constraint reads E_l sqrt(pT^2 + p_z^2) = mu + pz_l p_z; squared it is the
 * quadratic  a p_z^2 - 2 mu pz_l p_z + (E_l^2 pT^2 - mu^2) = 0  with
 * a = E_l^2 - pz_l^2, whose reduced discriminant is E_l^2 (mu^2 - a pT^2).
 * Roots (mu pz_l -/+ E_l sqrt(mu^2 - a pT^2)) / a; with a negative
 * discriminant the real part mu pz_l / a is the single candidate (reading).
 * Returns the candidate count (0 if a <= 0); kind[r] is 0/1 for the
 * minus/plus root, 2 for the real part.                                     */
int orc_nu_pz(const double l[4], double metx, double mety, double mw, double pz[2], int kind[2])
{
    double El = l[0], px = l[1], py = l[2], plz = l[3];
    double ml2 = El * El - px * px - py * py - plz * plz;
    double a = El * El - plz * plz;
    if (!(a > 0.0)) return 0;
    double pt2 = metx * metx + mety * mety;
    double mu = 0.5 * (mw * mw - ml2) + px * metx + py * mety;
    double d = mu * mu - a * pt2;
    if (d < 0.0) {
        pz[0] = mu * plz / a;
        kind[0] = 2;
        return 1;
    }
    double sq = El * sqrt(d);
    pz[0] = (mu * plz - sq) / a;
    pz[1] = (mu * plz + sq) / a;
    kind[0] = 0;
    kind[1] = 1;
    return 2;
}

static double orc_sq(double x) { return x * x; }

int64_t orc_semilep_reco(const orc_events *ev, const int32_t *idx, int64_t S, const orc_semilep_params *p,
                         const orc_semilep_out *out, int n_threads)
{
    int64_t npass = 0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : npass)
#endif
    for (int64_t s = 0; s < S; ++s) {
        int64_t e = (int64_t)idx[s] - ev->index_base;
        uint32_t l0 = ev->lep_off[e], l1 = ev->lep_off[e + 1];
        uint32_t j0 = ev->jet_off[e], j1 = ev->jet_off[e + 1];
        /* the lepton: the leading selected one (reading) */
        int64_t kl = -1;
        for (uint32_t k = l0; k < l1; ++k)
            if (orc_lep_sel(ev, k, p->lep_pt_min, p->lep_eta_max)) { kl = k; break; }
        /* jets: the selected ones in pT order, at most max_cands (reading) */
        int cap = p->max_cands < ORC_MAX_CANDS ? p->max_cands : ORC_MAX_CANDS;
        int cand[ORC_MAX_CANDS];
        vec4 cj[ORC_MAX_CANDS];
        int nc = 0;
        for (uint32_t k = j0; k < j1 && nc < cap; ++k)
            if (orc_jet_sel(ev, k, p->jet_pt_min, p->jet_eta_max)) {
                cand[nc] = (int)(k - j0);
                cj[nc] = orc_from_polar(ev->jet_pt[k], ev->jet_eta[k], ev->jet_phi[k], ev->jet_e[k]);
                ++nc;
            }
        int need = p->topology == ORC_TOPO_TCHAN ? 1 : p->topology == ORC_TOPO_WT ? 3 : 4;
        double pz[2];
        int kind[2];
        int nr = 0;
        vec4 lep = {0, 0, 0, 0};
        double mx = ev->met_x[e], my = ev->met_y[e];
        if (kl >= 0 && nc >= need) {
            lep = orc_from_polar(ev->lep_pt[kl], ev->lep_eta[kl], ev->lep_phi[kl], ev->lep_e[kl]);
            double l4[4] = {lep.e, lep.x, lep.y, lep.z};
            nr = orc_nu_pz(l4, mx, my, p->m_w, pz, kind);
        }
        int have = 0;
        double best = 0.0;
        int bj = -1, bh = -1, bp = -1, bq = -1, br = -1;
        double b_mtl = 0, b_mwl = 0, b_mth = ORC_NOSOL, b_mwh = ORC_NOSOL;
        vec4 b_nu = {0, 0, 0, 0};
        for (int r = 0; r < nr; ++r) {
            vec4 nu = {sqrt(mx * mx + my * my + pz[r] * pz[r]), mx, my, pz[r]};
            vec4 w = orc_add(lep, nu);
            double mwl = orc_mass(w);
            double c_w = orc_sq(mwl - p->m_w) / orc_sq(p->sigma_w);
            for (int j = 0; j < nc; ++j) {
                double mtl = orc_mass(orc_add(w, cj[j]));
                double c_t = orc_sq(mtl - p->m_t) / orc_sq(p->sigma_t);
                if (p->topology == ORC_TOPO_TCHAN) {
                    double chi2 = c_t + c_w;
                    if (!have || chi2 < best) {
                        have = 1; best = chi2; bj = j; br = r; b_mtl = mtl; b_mwl = mwl; b_nu = nu;
                    }
                    continue;
                }
                /* TTSEMI: every h; WT: no hadronic top (h = -1) */
                int nh = p->topology == ORC_TOPO_TTSEMI ? nc : 1;
                for (int hi = 0; hi < nh; ++hi) {
                    int h = p->topology == ORC_TOPO_TTSEMI ? hi : -1;
                    if (h == j) continue;
                    for (int a = 0; a < nc; ++a) {
                        if (a == j || a == h) continue;
                        for (int b = a + 1; b < nc; ++b) {
                            if (b == j || b == h) continue;
                            vec4 wh = orc_add(cj[a], cj[b]);
                            double mwh = orc_mass(wh);
                            double chi2 = c_t + c_w + orc_sq(mwh - p->m_w) / orc_sq(p->sigma_w);
                            double mth = ORC_NOSOL;
                            if (h >= 0) {
                                mth = orc_mass(orc_add(wh, cj[h]));
                                chi2 += orc_sq(mth - p->m_t) / orc_sq(p->sigma_t);
                            }
                            if (!have || chi2 < best) {
                                have = 1; best = chi2; bj = j; bh = h; bp = a; bq = b; br = r;
                                b_mtl = mtl; b_mwl = mwl; b_mth = mth; b_mwh = mwh; b_nu = nu;
                            }
                        }
                    }
                }
            }
        }
        out->has_sol[s] = (uint8_t)have;
        if (!have) {
            out->root[s] = -1;
            out->best_j[s] = out->best_h[s] = out->best_p[s] = out->best_q[s] = -1;
            for (int k = 0; k < 3; ++k) out->nu[3 * s + k] = ORC_NOSOL;
            out->m_tl[s] = out->m_wl[s] = out->m_th[s] = out->m_wh[s] = out->chi2[s] = ORC_NOSOL;
            continue;
        }
        ++npass;
        out->root[s] = (int8_t)kind[br];
        out->best_j[s] = (int16_t)cand[bj];
        out->best_h[s] = (int16_t)(bh >= 0 ? cand[bh] : -1);
        out->best_p[s] = (int16_t)(bp >= 0 ? cand[bp] : -1);
        out->best_q[s] = (int16_t)(bq >= 0 ? cand[bq] : -1);
        out->nu[3 * s + 0] = b_nu.x;
        out->nu[3 * s + 1] = b_nu.y;
        out->nu[3 * s + 2] = b_nu.z;
        out->m_tl[s] = b_mtl;
        out->m_wl[s] = b_mwl;
        out->m_th[s] = b_mth;
        out->m_wh[s] = b_mwh;
        out->chi2[s] = best;
    }
    return npass;
}

/* -------------------------------- dileptonic chi^2 fit with a MET split
 * Section 6.2: for the dileptonic final states the missing transverse
 * momentum is split between the two neutrinos and each neutrino's p_z then
 * follows from the mass constraints; the choice minimises Eq. (chi2) with
 * two tops (b l+ nu, bbar l- nubar) and two W (l+ nu, l- nubar).
 * Readings: the split is nu_T = MET/2 + (u, v), nubar_T = MET/2 - (u, v);
 * each p_z is the single-neutrino solution of orc_nu_pz (both roots, or the
 * real part); the minimum is searched on a square grid of (u, v) with
 * n_grid points per axis over [-half_range, half_range], then refined
 * n_refine times on a 5 x 5 grid centred on the best point so far with a
 * quarter of the previous step.  At every grid point every ordered pairing
 * of b candidates (i with l+, j with l-, i != j; candidates as in
 * orc_stage) and every pair of p_z candidates is scored; the first minimum
 * in the order (level, point, i, j, root of nu, root of nubar) is kept.
 * With one top (Wt: one top and two W bosons, section 6.2) each candidate
 * forms the top with l+ and then with l-, the other lepton's W standing
 * alone: Eq. (chi2) has that top's term and both W terms, and the first
 * minimum in the order (level, point, candidate, side, roots) is kept.     */

typedef struct {
    double m_t, m_w, sigma_t, sigma_w, half_range;
    double lep_pt_min, lep_eta_max, jet_pt_min, jet_eta_max, btag_min;
    int32_t pair_mode, max_cands, n_grid, n_refine, n_top;
} orc_chi2_params;

typedef struct {
    uint8_t *has_sol;
    int8_t *root_nu, *root_nubar;
    int16_t *best_i, *best_j;
    double *nu, *nubar; /* [S][3] */
    double *m_t, *m_tbar, *m_wp, *m_wm, *chi2, *split; /* split: [S][2] = (u, v) */
} orc_chi2_out;

typedef struct {
    double chi2, u, v;
    int i, j, r1, r2, have; /* one top: i or j is -1 on the side without it */
} orc_chi2_best;

/* chi^2 of every pairing and root pair at one split point; keeps the first
 * minimum in (i, j, r1, r2) order into *b when it beats b->chi2 strictly. */
static void orc_chi2_point(const orc_staged *st, double mx, double my, double u, double v,
                           const orc_chi2_params *p, orc_chi2_best *b)
{
    double n1x = 0.5 * mx + u, n1y = 0.5 * my + v;
    double n2x = 0.5 * mx - u, n2y = 0.5 * my - v;
    double lp[4] = {st->lp.e, st->lp.x, st->lp.y, st->lp.z};
    double lm[4] = {st->lm.e, st->lm.x, st->lm.y, st->lm.z};
    double pz1[2], pz2[2];
    int k1[2], k2[2];
    int n1 = orc_nu_pz(lp, n1x, n1y, p->m_w, pz1, k1);
    int n2 = orc_nu_pz(lm, n2x, n2y, p->m_w, pz2, k2);
    if (p->n_top == 1) {
        for (int i = 0; i < st->nc; ++i)
            for (int side = 0; side < 2; ++side)
                for (int r1 = 0; r1 < n1; ++r1)
                    for (int r2 = 0; r2 < n2; ++r2) {
                        vec4 nu = {sqrt(n1x * n1x + n1y * n1y + pz1[r1] * pz1[r1]), n1x, n1y, pz1[r1]};
                        vec4 nb = {sqrt(n2x * n2x + n2y * n2y + pz2[r2] * pz2[r2]), n2x, n2y, pz2[r2]};
                        vec4 wp = orc_add(st->lp, nu), wm = orc_add(st->lm, nb);
                        double mt = orc_mass(orc_add(st->cv[i], side == 0 ? wp : wm));
                        double chi2 = orc_sq(mt - p->m_t) / orc_sq(p->sigma_t) +
                                      orc_sq(orc_mass(wp) - p->m_w) / orc_sq(p->sigma_w) +
                                      orc_sq(orc_mass(wm) - p->m_w) / orc_sq(p->sigma_w);
                        if (!b->have || chi2 < b->chi2) {
                            b->have = 1; b->chi2 = chi2; b->u = u; b->v = v;
                            b->i = side == 0 ? i : -1; b->j = side == 0 ? -1 : i; b->r1 = r1; b->r2 = r2;
                        }
                    }
        return;
    }
    for (int i = 0; i < st->nc; ++i)
        for (int j = 0; j < st->nc; ++j) {
            if (i == j) continue;
            for (int r1 = 0; r1 < n1; ++r1)
                for (int r2 = 0; r2 < n2; ++r2) {
                    vec4 nu = {sqrt(n1x * n1x + n1y * n1y + pz1[r1] * pz1[r1]), n1x, n1y, pz1[r1]};
                    vec4 nb = {sqrt(n2x * n2x + n2y * n2y + pz2[r2] * pz2[r2]), n2x, n2y, pz2[r2]};
                    vec4 wp = orc_add(st->lp, nu), wm = orc_add(st->lm, nb);
                    double mt1 = orc_mass(orc_add(st->cv[i], wp));
                    double mt2 = orc_mass(orc_add(st->cv[j], wm));
                    double chi2 = orc_sq(mt1 - p->m_t) / orc_sq(p->sigma_t) + orc_sq(orc_mass(wp) - p->m_w) /
                                  orc_sq(p->sigma_w) + orc_sq(mt2 - p->m_t) / orc_sq(p->sigma_t) +
                                  orc_sq(orc_mass(wm) - p->m_w) / orc_sq(p->sigma_w);
                    if (!b->have || chi2 < b->chi2) {
                        b->have = 1; b->chi2 = chi2; b->u = u; b->v = v;
                        b->i = i; b->j = j; b->r1 = r1; b->r2 = r2;
                    }
                }
        }
}

int64_t orc_dilep_chi2_reco(const orc_events *ev, const int32_t *idx, int64_t S, const orc_chi2_params *p,
                            const orc_chi2_out *out, int n_threads)
{
    orc_reco_params rp;
    memset(&rp, 0, sizeof rp);
    rp.lep_pt_min = p->lep_pt_min; rp.lep_eta_max = p->lep_eta_max;
    rp.jet_pt_min = p->jet_pt_min; rp.jet_eta_max = p->jet_eta_max; rp.btag_min = p->btag_min;
    rp.pair_mode = p->pair_mode; rp.max_cands = p->max_cands;
    int64_t npass = 0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : npass)
#endif
    for (int64_t s = 0; s < S; ++s) {
        int64_t e = (int64_t)idx[s] - ev->index_base;
        orc_staged st;
        memset(&st, 0, sizeof st);
        if (e >= 0 && e < ev->n) st = orc_stage(ev, e, &rp);
        orc_chi2_best b;
        memset(&b, 0, sizeof b);
        double mx = 0.0, my = 0.0;
        /* one top needs one candidate, two tops two */
        if (p->n_top == 1 ? (st.leps && st.nc >= 1) : st.ok) {
            mx = ev->met_x[e];
            my = ev->met_y[e];
            /* coarse grid, then the refinements around the best point so far */
            double step = 2.0 * p->half_range / (double)(p->n_grid - 1);
            for (int a = 0; a < p->n_grid; ++a)
                for (int c = 0; c < p->n_grid; ++c)
                    orc_chi2_point(&st, mx, my, -p->half_range + step * a, -p->half_range + step * c, p, &b);
            for (int level = 0; level < p->n_refine && b.have; ++level) {
                step *= 0.25;
                double cu = b.u, cv = b.v;
                for (int a = -2; a <= 2; ++a)
                    for (int c = -2; c <= 2; ++c)
                        orc_chi2_point(&st, mx, my, cu + step * a, cv + step * c, p, &b);
            }
        }
        out->has_sol[s] = (uint8_t)b.have;
        if (!b.have) {
            out->root_nu[s] = out->root_nubar[s] = -1;
            out->best_i[s] = out->best_j[s] = -1;
            for (int k = 0; k < 3; ++k) out->nu[3 * s + k] = out->nubar[3 * s + k] = ORC_NOSOL;
            out->m_t[s] = out->m_tbar[s] = out->m_wp[s] = out->m_wm[s] = out->chi2[s] = ORC_NOSOL;
            out->split[2 * s] = out->split[2 * s + 1] = ORC_NOSOL;
            continue;
        }
        ++npass;
        /* the winner's kinematics */
        double n1x = 0.5 * mx + b.u, n1y = 0.5 * my + b.v, n2x = 0.5 * mx - b.u, n2y = 0.5 * my - b.v;
        double lp[4] = {st.lp.e, st.lp.x, st.lp.y, st.lp.z};
        double lm[4] = {st.lm.e, st.lm.x, st.lm.y, st.lm.z};
        double pz1[2], pz2[2];
        int k1[2], k2[2];
        orc_nu_pz(lp, n1x, n1y, p->m_w, pz1, k1);
        orc_nu_pz(lm, n2x, n2y, p->m_w, pz2, k2);
        vec4 nu = {sqrt(n1x * n1x + n1y * n1y + pz1[b.r1] * pz1[b.r1]), n1x, n1y, pz1[b.r1]};
        vec4 nb = {sqrt(n2x * n2x + n2y * n2y + pz2[b.r2] * pz2[b.r2]), n2x, n2y, pz2[b.r2]};
        out->root_nu[s] = (int8_t)k1[b.r1];
        out->root_nubar[s] = (int8_t)k2[b.r2];
        out->best_i[s] = (int16_t)(b.i >= 0 ? st.cand[b.i] : -1);
        out->best_j[s] = (int16_t)(b.j >= 0 ? st.cand[b.j] : -1);
        out->nu[3 * s + 0] = nu.x; out->nu[3 * s + 1] = nu.y; out->nu[3 * s + 2] = nu.z;
        out->nubar[3 * s + 0] = nb.x; out->nubar[3 * s + 1] = nb.y; out->nubar[3 * s + 2] = nb.z;
        out->m_wp[s] = orc_mass(orc_add(st.lp, nu));
        out->m_wm[s] = orc_mass(orc_add(st.lm, nb));
        out->m_t[s] = b.i >= 0 ? orc_mass(orc_add(st.cv[b.i], orc_add(st.lp, nu))) : ORC_NOSOL;
        out->m_tbar[s] = b.j >= 0 ? orc_mass(orc_add(st.cv[b.j], orc_add(st.lm, nb))) : ORC_NOSOL;
        out->chi2[s] = b.chi2;
        out->split[2 * s] = b.u;
        out->split[2 * s + 1] = b.v;
    }
    return npass;
}
