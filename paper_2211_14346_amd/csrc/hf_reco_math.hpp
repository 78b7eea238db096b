// Device math of the two-neutrino reconstruction (paper section 4: W and top
// mass constraints per lepton / b-jet pairing).
//
// For a lepton l and a b jet b, the conditions (l+nu)^2 = mW^2 and
// (b+l+nu)^2 = mt^2 with a massless neutrino are linear in (E, pz) of the
// neutrino for given (px, py) = (x, y):
//     El E - lz pz = kl + lx x + ly y,      kl = (mW^2 - ml^2)/2
//     Eb E - bz pz = kb + bx x + by y,      kb = (mt^2 - mW^2 - mb^2 - 2 b.l)/2
// Their solution E = e1 x + e2 y + e0, pz = z1 x + z2 y + z0 turns the mass
// shell E^2 = x^2 + y^2 + pz^2 into a conic in (x, y).
//
// Scaling l by s_l and b by s_b (the resolution variations) leaves e1, e2,
// z1, z2 and the quadratic part of the conic unchanged; only
//     e0 = (lz/D) U - (bz/D) W,   pz0 = (El/D) U - (Eb/D) W,   D = lz Eb - El bz
// with U = kb'/s_b = (mt^2 - mW^2)/(2 s_b) - s_b mb^2/2 - s_l b.l and
// W = kl'/s_l = mW^2/(2 s_l) - s_l ml^2/2 move.  The per-candidate constants
// are therefore staged once per event and each variation costs a handful of
// FMAs before the quartic assembly.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

// Host-and-device so that the numerics can also be exercised on the CPU.
#define HF_HD __host__ __device__
#ifndef HF_ITER_HOOK
#define HF_ITER_HOOK()
#endif

namespace hf {

// 1/d to full FP64 precision from the hardware estimate plus two Newton
// refinements (the IEEE-exact division sequence is not needed where the
// result only steers an iteration or ranks candidates).
HF_HD __forceinline__ double fast_rcp(double d) {
#ifdef __HIP_DEVICE_COMPILE__
    double r = __builtin_amdgcn_rcp(d);
    r = fma(fma(-d, r, 1.0), r, r);
    r = fma(fma(-d, r, 1.0), r, r);
    return r;
#else
    return 1.0 / d;
#endif
}

// 1/d to about 2^-46 relative (the hardware estimate, good to about 2^-23,
// plus one Newton refinement), where the result only scales a correction
// step or a residual ratio: an error there changes the step taken, not the
// point the iteration converges to.
HF_HD __forceinline__ double step_rcp(double d) {
#ifdef __HIP_DEVICE_COMPILE__
    const double r = __builtin_amdgcn_rcp(d);
    return fma(fma(-d, r, 1.0), r, r);
#else
    return 1.0 / d;
#endif
}

// sqrt(v) for v >= 0 to about one ulp: the hardware reciprocal square root
// and one Goldschmidt refinement (no IEEE correction sequence).
HF_HD __forceinline__ double fast_sqrt(double v) {
#ifdef __HIP_DEVICE_COMPILE__
    if (!(v > 0.0)) return 0.0;
    const double y = __builtin_amdgcn_rsq(v);
    double s = v * y, h = 0.5 * y;
    const double r = fma(-s, h, 0.5);
    s = fma(s, r, s);
    h = fma(h, r, h);
    const double d = fma(-s, s, v);
    return fma(d, h, s);
#else
    return sqrt(v);
#endif
}

// constants of one (lepton, b candidate) side, nominal kinematics
enum SideField { kE1 = 0, kE2, kZ1, kZ2, kAl, kBe, kGa, kDe, kQxx, kQxy, kQyy, kMb2, kBl, kSide };

// Bivariate quadratic  xx x^2 + xy x y + yy y^2 + x x + y y + c.
struct Conic {
    double xx, xy, yy, x, y, c;
};

HF_HD __forceinline__ double conic_eval(const Conic &q, double x, double y) {
    return fma(x, fma(q.xx, x, fma(q.xy, y, q.x)), fma(y, fma(q.yy, y, q.y), q.c));
}

HF_HD __forceinline__ double conic_mag(const Conic &q, double x, double y) {
    return fabs(q.xx * x * x) + fabs(q.xy * x * y) + fabs(q.yy * y * y) + fabs(q.x * x) + fabs(q.y * y) +
           fabs(q.c);
}

// Side constants from nominal 4-vectors (E, px, py, pz); returns false when
// the 2x2 system is degenerate: |D| <= 1e-5 El Eb (for massless l and b their
// direction cosines along the beam agree to 1e-5; the map's coefficients grow
// as 1/D, the mass shell's rounding faster, and FP64 no longer resolves the
// constraints below that).  The test is invariant under scaling.
HF_HD __forceinline__ bool make_side(const double l[4], const double b[4], double s[kSide]) {
    const double D = l[3] * b[0] - l[0] * b[3];
    if (!(fabs(D) > 1e-5 * l[0] * b[0])) {
        for (int k = 0; k < kSide; ++k) s[k] = 0.0;
        return false;
    }
    const double inv = 1.0 / D;
    const double e1 = (l[3] * b[1] - b[3] * l[1]) * inv;
    const double e2 = (l[3] * b[2] - b[3] * l[2]) * inv;
    const double z1 = (l[0] * b[1] - b[0] * l[1]) * inv;
    const double z2 = (l[0] * b[2] - b[0] * l[2]) * inv;
    s[kE1] = e1;
    s[kE2] = e2;
    s[kZ1] = z1;
    s[kZ2] = z2;
    s[kAl] = l[3] * inv;
    s[kBe] = b[3] * inv;
    s[kGa] = l[0] * inv;
    s[kDe] = b[0] * inv;
    s[kQxx] = e1 * e1 - 1.0 - z1 * z1;
    s[kQxy] = 2.0 * (e1 * e2 - z1 * z2);
    s[kQyy] = e2 * e2 - 1.0 - z2 * z2;
    s[kMb2] = b[0] * b[0] - b[1] * b[1] - b[2] * b[2] - b[3] * b[3];
    s[kBl] = b[0] * l[0] - b[1] * l[1] - b[2] * l[2] - b[3] * l[3];
    return true;
}

// Varying part of one side for scale factors (s_l, s_b): e0, pz0 and the
// conic's linear and constant coefficients.
struct SideVar {
    double e0, z0;
    Conic q;
};

HF_HD __forceinline__ SideVar side_var(const double *s, double W, double s_l, double s_b, double mt2_mw2) {
    SideVar r;
    const double U = (0.5 * mt2_mw2) * fast_rcp(s_b) - 0.5 * s_b * s[kMb2] - s_l * s[kBl];
    r.e0 = s[kAl] * U - s[kBe] * W;
    r.z0 = s[kGa] * U - s[kDe] * W;
    r.q.xx = s[kQxx];
    r.q.xy = s[kQxy];
    r.q.yy = s[kQyy];
    r.q.x = 2.0 * (s[kE1] * r.e0 - s[kZ1] * r.z0);
    r.q.y = 2.0 * (s[kE2] * r.e0 - s[kZ2] * r.z0);
    r.q.c = r.e0 * r.e0 - r.z0 * r.z0;
    return r;
}

// q(mx - x, my - y) as a conic in (x, y).
HF_HD __forceinline__ Conic reflect(const Conic &q, double mx, double my) {
    Conic r;
    r.xx = q.xx;
    r.xy = q.xy;
    r.yy = q.yy;
    r.x = -2.0 * q.xx * mx - q.xy * my - q.x;
    r.y = -q.xy * mx - 2.0 * q.yy * my - q.y;
    r.c = mx * (q.xx * mx + q.xy * my + q.x) + my * (q.yy * my + q.y) + q.c;
    return r;
}

// Eliminant in y of the two conics, written as P(y) = a y^2 + b(x) y + c(x)
// and Q(y) = d y^2 + e(x) y + f(x): Res = (a f - c d)^2 - (a e - b d)(b f - c e),
// a quartic in x.  Coefficients ascending in x.
HF_HD __forceinline__ void eliminant(const Conic &P, const Conic &Q, double q[5]) {
    const double a = P.yy, b1 = P.xy, b0 = P.y, c2 = P.xx, c1 = P.x, c0 = P.c;
    const double d = Q.yy, e1 = Q.xy, e0 = Q.y, f2 = Q.xx, f1 = Q.x, f0 = Q.c;
    const double g2 = a * f2 - d * c2, g1 = a * f1 - d * c1, g0 = a * f0 - d * c0;
    const double h1 = a * e1 - d * b1, h0 = a * e0 - d * b0;
    const double k3 = b1 * f2 - c2 * e1;
    const double k2 = b1 * f1 + b0 * f2 - c2 * e0 - c1 * e1;
    const double k1 = b1 * f0 + b0 * f1 - c1 * e0 - c0 * e1;
    const double k0 = b0 * f0 - c0 * e0;
    q[4] = g2 * g2 - h1 * k3;
    q[3] = 2.0 * g2 * g1 - h1 * k2 - h0 * k3;
    q[2] = g1 * g1 + 2.0 * g2 * g0 - h1 * k1 - h0 * k2;
    q[1] = 2.0 * g1 * g0 - h1 * k0 - h0 * k1;
    q[0] = g0 * g0 - h0 * k0;
}

// ------------------------------------------------------------------ roots
// Real roots of the quartic by critical points: the critical points (roots
// of the derivative) come from the closed-form cubic in precision T and are
// polished once in FP64; every monotone interval whose end values differ in
// sign is then solved by Halley's method in FP64, safeguarded by bisection.
// Like the oracle, the polynomial is taken in t = x / 100 GeV, normalised by
// its largest coefficient, and coefficients <= 1e-14 are dropped from the top.

constexpr double kXScale = 100.0;

// Quartic and its first two derivatives with all five coefficients (dropped
// leading coefficients are zero), so that no register array is indexed at
// run time.
struct Poly4 {
    double c0, c1, c2, c3, c4;
};

HF_HD __forceinline__ double peval(const Poly4 &c, double t) {
    return fma(fma(fma(fma(c.c4, t, c.c3), t, c.c2), t, c.c1), t, c.c0);
}

HF_HD __forceinline__ void peval_d(const Poly4 &c, double t, double &p, double &dp) {
    p = peval(c, t);
    dp = fma(fma(fma(4.0 * c.c4, t, 3.0 * c.c3), t, 2.0 * c.c2), t, c.c1);
}

HF_HD __forceinline__ double peval_d1(const Poly4 &c, double t) {
    return fma(fma(fma(4.0 * c.c4, t, 3.0 * c.c3), t, 2.0 * c.c2), t, c.c1);
}

HF_HD __forceinline__ double peval_d2(const Poly4 &c, double t) {
    return fma(fma(12.0 * c.c4, t, 6.0 * c.c3), t, 2.0 * c.c2);
}

// Elementary functions for the templated cubic.  FP64: the accurate library
// functions.  FP32 (seeds only, refined in FP64 afterwards): hardware
// approximations -- square root and reciprocal by the single-instruction
// units (about one ulp, no correction sequence), cube root through the base-2
// exponential and logarithm units, arc cosine by the four-term approximation
// of Abramowitz & Stegun 4.4.45 (|error| < 7e-5 rad), cosine/sine through the
// revolution-scaled hardware units.
HF_HD __forceinline__ float tsqrt(float v) {
#ifdef __HIP_DEVICE_COMPILE__
    return __builtin_amdgcn_sqrtf(v);
#else
    return sqrtf(v);
#endif
}
HF_HD __forceinline__ double tsqrt(double v) { return sqrt(v); }
HF_HD __forceinline__ float trcp(float v) {
#ifdef __HIP_DEVICE_COMPILE__
    return __builtin_amdgcn_rcpf(v);
#else
    return 1.0f / v;
#endif
}
HF_HD __forceinline__ double trcp(double v) { return 1.0 / v; }
HF_HD __forceinline__ double tcbrt(double v) { return cbrt(v); }
HF_HD __forceinline__ float tcbrt(float v) {
#ifdef __HIP_DEVICE_COMPILE__
    const float m = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(fabsf(v)) * (1.0f / 3.0f));
#else
    const float m = exp2f(log2f(fabsf(v)) * (1.0f / 3.0f));
#endif
    return v == 0.0f ? 0.0f : copysignf(m, v);
}
HF_HD __forceinline__ double tacos(double v) { return acos(v); }
HF_HD __forceinline__ float tacos(float x) {
    const float ax = fabsf(x);
    const float r = sqrtf(1.0f - ax) * (1.5707288f + ax * (-0.2121144f + ax * (0.0742610f - 0.0187293f * ax)));
    return x < 0.0f ? 3.14159265358979f - r : r;
}
HF_HD __forceinline__ void tsincos(double a, double &s, double &c) {
    s = sin(a);
    c = cos(a);
}
HF_HD __forceinline__ void tsincos(float a, float &s, float &c) {
#ifdef __HIP_DEVICE_COMPILE__
    const float rev = a * 0.15915494309189535f;  // radians -> revolutions
    s = __builtin_amdgcn_sinf(rev);
    c = __builtin_amdgcn_cosf(rev);
#else
    s = sinf(a);
    c = cosf(a);
#endif
}
HF_HD __forceinline__ float tmin(float a, float b) { return fminf(a, b); }
HF_HD __forceinline__ double tmin(double a, double b) { return fmin(a, b); }
HF_HD __forceinline__ float tmax(float a, float b) { return fmaxf(a, b); }
HF_HD __forceinline__ double tmax(double a, double b) { return fmax(a, b); }

// Real roots (ascending) of the monic cubic s^3 + A s^2 + B s + C in
// precision T; returns 1 or 3.
template <typename T>
HF_HD __forceinline__ int cubic_roots(T A, T B, T C, T &r0, T &r1, T &r2) {
    const T third = (T)(1.0 / 3.0);
    const T a3 = A * third;
    const T p = B - A * a3;  // depressed: u^3 + p u + q
    const T q = (T)2 * a3 * a3 * a3 - a3 * B + C;
    const T h = (T)0.5 * q;
    const T p3 = p * third;
    const T disc = h * h + p3 * p3 * p3;
    if (disc > (T)0) {
        const T sq = tsqrt(disc);
        const T w = -h - (h >= (T)0 ? sq : -sq);
        const T u = tcbrt(w);
        const T r = (u != (T)0) ? u - p3 * trcp(u) : (T)0;
        r0 = r1 = r2 = r - a3;
        return 1;
    }
    const T rr = tsqrt(tmax(-p3, (T)0));
    T cosarg = (rr > (T)0) ? -h * trcp(rr * rr * rr) : (T)0;
    cosarg = tmin(tmax(cosarg, (T)-1), (T)1);
    const T phi = tacos(cosarg) * third;
    T sn, cs;
    tsincos(phi, sn, cs);
    // cos(phi -+ 2 pi / 3) = -cos(phi) / 2 +- sin(phi) sqrt(3) / 2
    const T h3 = (T)0.86602540378443865 * sn;
    const T x0 = (T)2 * rr * cs - a3;                        // largest
    const T x1 = (T)2 * rr * ((T)-0.5 * cs + h3) - a3;       // middle
    const T x2 = (T)2 * rr * ((T)-0.5 * cs - h3) - a3;       // smallest
    r0 = tmin(tmin(x0, x1), x2);
    r2 = tmax(tmax(x0, x1), x2);
    r1 = x0 + x1 + x2 - r0 - r2;
    return 3;
}

// Root of c on (lo, hi) where c(lo) < 0 iff lo_neg; x is the first iterate.
// Halley's step  dx = p p' / (p'^2 - p p'' / 2)  (cubic convergence, so a
// wavefront's slowest lane needs fewer iterations), taken as the Newton step
// p / p' wherever Halley's correction factor p'^2 / (p'^2 - p p'' / 2) leaves
// (1/2, 2), i.e. far from the root; steps that leave the bracket are replaced
// by bisection.  Converged when the step is below 1e-12 max(1, |t|) (t = x /
// 100 GeV), or below 1e-7 max(1, |t|) and 1e-3 of the previous step (the
// error after that step is far below its size).  The test comes before the
// bracket update so that an iterate sitting on a bracket end at convergence
// is not bisected away.  A root next to a critical point (a near double root)
// is fixed only to the polynomial's rounding, where the step tests can fail
// forever: from the sixth iterate on, the search also stops when |p| is at
// its rounding floor (1e-15 of the sum of its terms' magnitudes) or the
// bracket is narrower than the tolerance.
HF_HD __forceinline__ double bracket_halley(const Poly4 &c, double lo, double hi, bool lo_neg, double x) {
    double dx_prev = 0.0;
    for (int it = 0; it < 60; ++it) {
        HF_ITER_HOOK();
        double p, dp;
        peval_d(c, x, p, dp);
        if (p == 0.0) return x;
        if ((p < 0.0) == lo_neg)
            lo = x;
        else
            hi = x;
        const double d2 = peval_d2(c, x);
        const double g = dp * dp;
        const double hd = fma(-0.5 * p, d2, g);
        const double den = (hd > 0.5 * g && hd < 2.0 * g) ? hd : g;
        const double dx = p * dp * step_rcp(den);
        const double tol = 1e-12 * fmax(1.0, fabs(x));
        if (fabs(dx) <= tol) return x - dx;
        if (it >= 1 && fabs(dx) <= 1e5 * tol && fabs(dx) <= 1e-3 * fabs(dx_prev)) return x - dx;
        if (it >= 5) {
            // slow convergence (a root next to a critical point): stop once p is
            // at its rounding floor or the bracket is below the tolerance
            const double ax = fabs(x);
            const double mag =
                (((fabs(c.c4) * ax + fabs(c.c3)) * ax + fabs(c.c2)) * ax + fabs(c.c1)) * ax + fabs(c.c0);
            if (fabs(p) <= 1e-15 * mag || hi - lo <= tol) return x;
        }
        double xn = x - dx;
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        dx_prev = dx;
        x = xn;
    }
    return x;
}

// Root of the interval [lo, hi] (values flo, fhi of opposite signs), in x
// units.  First iterate: the quadratic model p(e + d) ~ p(e) + p''(e) d^2 / 2
// at a critical end e -- for an interval between two critical points, at the
// end where |p| is smaller (the root lies nearer to it), with the secant as
// the fallback.
HF_HD __forceinline__ void solve_interval(const Poly4 &c, double lo, double hi, double flo, double fhi, bool lo_crit,
                                          bool hi_crit, double &root, bool &found) {
    found = false;
    if (!((flo < 0.0 && fhi > 0.0) || (flo > 0.0 && fhi < 0.0)) || !(hi > lo)) return;
    double x0;
    if (lo_crit || hi_crit) {
        const bool from_lo = lo_crit && (!hi_crit || fabs(flo) <= fabs(fhi));
        const double cp = from_lo ? lo : hi;
        const double fv = from_lo ? flo : fhi;
        const double r = -2.0 * fv * step_rcp(peval_d2(c, cp));
        if (r > 0.0)
            x0 = from_lo ? cp + fast_sqrt(r) : cp - fast_sqrt(r);
        else
            x0 = (lo_crit && hi_crit) ? lo : from_lo ? cp + fmax(1.0, fabs(cp)) : cp - fmax(1.0, fabs(cp));
        if (lo_crit && hi_crit && !(x0 > lo && x0 < hi)) x0 = lo - flo * (hi - lo) * step_rcp(fhi - flo);
    } else {
        x0 = 0.0;
    }
    if (!(x0 > lo && x0 < hi)) x0 = 0.5 * (lo + hi);
    root = kXScale * bracket_halley(c, lo, hi, flo < 0.0, x0);
    found = true;
}

// Sign-changing real roots of q0 + q1 x + ... + q4 x^4 by critical points:
// the roots of the derivative (closed-form cubic in precision T, one FP64
// Newton step each) split the line into monotone intervals; each interval
// whose end values differ in sign holds one root, found by safeguarded
// Halley iteration in FP64.  As in the oracle, the polynomial is taken in t = x / 100 GeV,
// normalised by its largest coefficient, and leading coefficients <= 1e-14
// are dropped; the outer intervals end at the Cauchy bound.
//
// quartic_brackets does everything up to the intervals; bracket_root solves
// one interval.  The search kernel runs the two on different lanes.
struct Brackets {
    Poly4 c;             // normalised polynomial in t
    double e1, e2, e3;   // inner interval ends (critical points); direct roots for degree <= 2
    double bound;        // intervals are [-bound, e1], [e1, e2], [e2, e3], [e3, bound]
    double f1, f2, f3;   // polynomial values at e1, e2, e3
    int mask;            // bit k: interval k holds a root (or: direct root k exists)
    int direct;          // 1: degree <= 2, roots given directly in e1, e2
    int signs;           // bit 0: p(-bound) < 0; bit 1: p(+bound) < 0
};

template <typename T>
HF_HD __forceinline__ Brackets quartic_brackets(const double qx[5]) {
    Brackets B;
    B.mask = 0;
    B.direct = 0;
    B.signs = 0;
    B.e1 = B.e2 = B.e3 = B.f1 = B.f2 = B.f3 = 0.0;
    B.bound = 1.0;
    Poly4 &c = B.c;
    c = Poly4{qx[0], qx[1] * kXScale, qx[2] * (kXScale * kXScale), qx[3] * (kXScale * kXScale * kXScale),
              qx[4] * (kXScale * kXScale * kXScale * kXScale)};
    const double mx = fmax(fmax(fmax(fabs(c.c0), fabs(c.c1)), fmax(fabs(c.c2), fabs(c.c3))), fabs(c.c4));
    if (!(mx > 0.0) || !isfinite(mx)) return B;
    const double inv = fast_rcp(mx);
    c.c0 *= inv;
    c.c1 *= inv;
    c.c2 *= inv;
    c.c3 *= inv;
    c.c4 *= inv;
    int n = 4;
    if (fabs(c.c4) <= 1e-14) {
        c.c4 = 0.0;
        n = 3;
        if (fabs(c.c3) <= 1e-14) {
            c.c3 = 0.0;
            n = 2;
            if (fabs(c.c2) <= 1e-14) {
                c.c2 = 0.0;
                n = 1;
                if (fabs(c.c1) <= 1e-14) return B;
            }
        }
    }
    if (n <= 2) {
        B.direct = 1;
        if (n == 1) {
            B.e1 = -c.c0 / c.c1;
            B.mask = 1;
        } else {
            const double disc = c.c1 * c.c1 - 4.0 * c.c2 * c.c0;
            if (disc > 0.0) {
                const double sq = sqrt(disc);
                const double t = -0.5 * (c.c1 + (c.c1 >= 0.0 ? sq : -sq));
                const double a = t / c.c2, b = c.c0 / t;
                B.e1 = fmin(a, b);
                B.e2 = fmax(a, b);
                B.mask = 3;
            }
        }
        return B;
    }
    const double lead = n == 4 ? c.c4 : c.c3;
    const double il = fast_rcp(lead);
    double bound = fmax(fmax(fabs(c.c0 * il), fabs(c.c1 * il)), fabs(c.c2 * il));
    if (n == 4) bound = fmax(bound, fabs(c.c3 * il));
    bound += 1.0;
    // critical points k0 <= k1 <= k2 (nk of them)
    double k0 = 0.0, k1 = 0.0, k2 = 0.0;
    int nk = 0;
    if (n == 4) {
        const double A = 0.75 * c.c3 * il, Bc = 0.5 * c.c2 * il, C = 0.25 * c.c1 * il;
        if (fmax(fabs(A), fmax(fabs(Bc), fabs(C))) < 1e6) {
            T a0, a1, a2;
            nk = cubic_roots<T>((T)A, (T)Bc, (T)C, a0, a1, a2);
            k0 = (double)a0;
            k1 = (double)a1;
            k2 = (double)a2;
        } else {
            nk = cubic_roots<double>(A, Bc, C, k0, k1, k2);
        }
    } else {  // n == 3: derivative 3 c3 t^2 + 2 c2 t + c1
        const double a = 3.0 * c.c3, b = 2.0 * c.c2, cc = c.c1;
        const double disc = b * b - 4.0 * a * cc;
        if (disc > 0.0) {
            const double sq = sqrt(disc);
            const double t = -0.5 * (b + (b >= 0.0 ? sq : -sq));
            const double r1 = t / a, r2 = cc / t;
            k0 = fmin(r1, r2);
            k1 = fmax(r1, r2);
            nk = 2;
        }
    }
    // one FP64 Newton step on the derivative for each critical point
    {
        double g, gp;
        g = peval_d1(c, k0);
        gp = peval_d2(c, k0);
        if (gp != 0.0) k0 -= g * step_rcp(gp);
        g = peval_d1(c, k1);
        gp = peval_d2(c, k1);
        if (gp != 0.0) k1 -= g * step_rcp(gp);
        g = peval_d1(c, k2);
        gp = peval_d2(c, k2);
        if (gp != 0.0) k2 -= g * step_rcp(gp);
    }
    // interval ends -B, k0, k1, k2, B; missing or out-of-range critical points
    // collapse onto +B, which empties their intervals
    const bool pos_hi = lead > 0.0;
    const bool neg_lo = (n & 1) ? pos_hi : !pos_hi;  // p(-B) < 0
    const bool u0 = nk >= 1 && k0 > -bound && k0 < bound;
    const bool u1 = nk >= 2 && k1 > -bound && k1 < bound;
    const bool u2 = nk >= 3 && k2 > -bound && k2 < bound;
    double e1 = u0 ? k0 : bound, e2 = u1 ? k1 : bound, e3 = u2 ? k2 : bound;
    if (e2 < e1) { const double t = e1; e1 = e2; e2 = t; }
    if (e3 < e2) { const double t = e2; e2 = e3; e3 = t; }
    if (e2 < e1) { const double t = e1; e1 = e2; e2 = t; }
    const double sb = pos_hi ? 1.0 : -1.0;
    const double f0 = neg_lo ? -1.0 : 1.0;
    const double f1 = e1 < bound ? peval(c, e1) : sb;
    const double f2 = e2 < bound ? peval(c, e2) : sb;
    const double f3 = e3 < bound ? peval(c, e3) : sb;
    B.e1 = e1;
    B.e2 = e2;
    B.e3 = e3;
    B.bound = bound;
    B.f1 = f1;
    B.f2 = f2;
    B.f3 = f3;
    B.signs = (neg_lo ? 1 : 0) | (pos_hi ? 0 : 2);
    auto change = [](double a, double b, double lo, double hi) {
        return ((a < 0.0 && b > 0.0) || (a > 0.0 && b < 0.0)) && hi > lo;
    };
    B.mask = (change(f0, f1, -bound, e1) ? 1 : 0) | (change(f1, f2, e1, e2) ? 2 : 0) |
             (change(f2, f3, e2, e3) ? 4 : 0) | (change(f3, sb, e3, bound) ? 8 : 0);
    return B;
}

// Root (in t units) in interval k of a Brackets record, or direct root k.
HF_HD __forceinline__ double bracket_root(const Brackets &B, int k) {
    if (B.direct) return k == 0 ? B.e1 : B.e2;
    const double lo = k == 0 ? -B.bound : k == 1 ? B.e1 : k == 2 ? B.e2 : B.e3;
    const double hi = k == 0 ? B.e1 : k == 1 ? B.e2 : k == 2 ? B.e3 : B.bound;
    const double f0 = (B.signs & 1) ? -1.0 : 1.0, f4 = (B.signs & 2) ? -1.0 : 1.0;
    const double flo = k == 0 ? f0 : k == 1 ? B.f1 : k == 2 ? B.f2 : B.f3;
    const double fhi = k == 0 ? B.f1 : k == 1 ? B.f2 : k == 2 ? B.f3 : f4;
    const bool lo_crit = k > 0 && lo < B.bound;
    const bool hi_crit = k < 3 && hi < B.bound;
    double root = 0.0;
    bool found;
    solve_interval(B.c, lo, hi, flo, fhi, lo_crit, hi_crit, root, found);
    return root * (1.0 / kXScale);  // solve_interval returns x units
}

// Sign-changing real roots (in x units), ascending in slots 0 .. popcount(mask) - 1.
struct Roots4 {
    double r[4];
    int mask;
};

HF_HD __forceinline__ double pick4(const double r[4], int k) {
    return k == 0 ? r[0] : k == 1 ? r[1] : k == 2 ? r[2] : r[3];
}

template <typename T>
HF_HD Roots4 quartic_real_roots(const double qx[5]) {
    const Brackets B = quartic_brackets<T>(qx);
    Roots4 out;
    out.r[0] = out.r[1] = out.r[2] = out.r[3] = 0.0;
    int nb = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (!((B.mask >> k) & 1)) continue;
        const double x = kXScale * bracket_root(B, k);
        out.r[0] = nb == 0 ? x : out.r[0];
        out.r[1] = nb == 1 ? x : out.r[1];
        out.r[2] = nb == 2 ? x : out.r[2];
        out.r[3] = nb == 3 ? x : out.r[3];
        ++nb;
    }
    out.mask = (1 << nb) - 1;
    return out;
}

// y of an intersection at abscissa x.  The elimination a Q - d P is linear
// in y; when its coefficient is not small against its terms that gives y
// directly.  Otherwise (two intersections sharing nearly the same x) the
// candidates are the elimination and the real roots of P and of Q in y, and
// the one with the smallest sum of relative residuals wins.  Returns false
// if there is no candidate.
HF_HD __forceinline__ bool recover_y(const Conic &P, const Conic &Q, double x, double &y) {
    const double a = P.yy, bx = fma(P.xy, x, P.y), cx = fma(fma(P.xx, x, P.x), x, P.c);
    const double d = Q.yy, ex = fma(Q.xy, x, Q.y), fx = fma(fma(Q.xx, x, Q.x), x, Q.c);
    const double den = bx * d - a * ex;
    if (fabs(den) > 1e-3 * (fabs(bx * d) + fabs(a * ex))) {
        y = (a * fx - cx * d) * fast_rcp(den);
        return true;
    }
    // slow path: five fixed candidate slots with validity flags
    double best = INFINITY;
    bool any = false;
    auto consider = [&](double yy) {
        const double rp = fabs(fma(fma(a, yy, bx), yy, cx)) * fast_rcp(fabs(a) * yy * yy + fabs(bx * yy) + fabs(cx));
        const double rq = fabs(fma(fma(d, yy, ex), yy, fx)) * fast_rcp(fabs(d) * yy * yy + fabs(ex * yy) + fabs(fx));
        const double r = rp + rq;
        if (!any || r < best) {
            best = r;
            y = yy;
            any = true;
        }
    };
    if (den != 0.0) consider((a * fx - cx * d) / den);
    auto quad = [&](double A, double Bq, double C) {
        if (A == 0.0) {
            if (Bq != 0.0) consider(-C / Bq);
            return;
        }
        const double disc = Bq * Bq - 4.0 * A * C;
        if (disc < 0.0) return;
        const double sq = sqrt(disc);
        const double t = -0.5 * (Bq + (Bq >= 0.0 ? sq : -sq));
        if (t == 0.0) {
            consider(0.0);
            return;
        }
        consider(t / A);
        consider(C / t);
    };
    quad(a, bx, cx);
    quad(d, ex, fx);
    return any;
}

// Acceptance of an intersection (section 4 constraints).  The W and top
// constraints hold by construction of the linear maps, and each conic's value
// is that neutrino's squared mass E^2 - p^2 in GeV^2, which is also the offset
// of (l + nu)^2 from mW^2 and of (b + l + nu)^2 from mt^2.  A point is a
// solution when both squared masses are within kAcceptM2 mW^2 of zero: every
// mass constraint then holds to 1e-6 relative.
constexpr double kAcceptM2 = 2e-6;

// Points whose squared masses are already 100 times inside the acceptance
// bound (every mass within 1e-8 relative) are not polished.
constexpr double kPolishSkip = 1e-2;

// Newton's method on the two conics for (x, y), each step kept only while it
// lowers the larger relative residual (|value| over the sum of the magnitudes
// of the conic's terms).  Returns max(|P(x, y)|, |Q(x, y)|) in GeV^2 at the
// final point; skip_below: no step is taken from a point already below it.
HF_HD __forceinline__ double polish_xy(const Conic &P, const Conic &Q, double &x, double &y, int iters,
                                       double skip_below) {
    double f1 = conic_eval(P, x, y), f2 = conic_eval(Q, x, y);
    double phys = fmax(fabs(f1), fabs(f2));
    if (!(phys > skip_below)) return phys;
    double res = fmax(fabs(f1) * step_rcp(conic_mag(P, x, y)), fabs(f2) * step_rcp(conic_mag(Q, x, y)));
    for (int it = 0; it < iters; ++it) {
        if (res == 0.0) break;
        const double a11 = 2.0 * P.xx * x + P.xy * y + P.x, a12 = P.xy * x + 2.0 * P.yy * y + P.y;
        const double a21 = 2.0 * Q.xx * x + Q.xy * y + Q.x, a22 = Q.xy * x + 2.0 * Q.yy * y + Q.y;
        const double det = a11 * a22 - a12 * a21;
        if (det == 0.0) break;
        const double id = step_rcp(det);
        const double xn = x + (-f1 * a22 + f2 * a12) * id;
        const double yn = y + (-a11 * f2 + a21 * f1) * id;
        const double g1 = conic_eval(P, xn, yn), g2 = conic_eval(Q, xn, yn);
        const double rn = fmax(fabs(g1) * step_rcp(conic_mag(P, xn, yn)), fabs(g2) * step_rcp(conic_mag(Q, xn, yn)));
        if (!(rn < res)) break;
        x = xn;
        y = yn;
        f1 = g1;
        f2 = g2;
        res = rn;
        phys = fmax(fabs(f1), fabs(f2));
        if (!(phys > skip_below)) break;
    }
    return phys;
}

}  // namespace hf
