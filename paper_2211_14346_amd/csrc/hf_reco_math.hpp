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
// FMAs before the two conics are intersected.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

// Host-and-device so that the numerics can also be exercised on the CPU.
#define HF_HD __host__ __device__

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

// 1/sqrt(v) for v > 0 to about 2^-46 relative: the hardware estimate and one
// Newton refinement.
HF_HD __forceinline__ double step_rsqrt(double v) {
#ifdef __HIP_DEVICE_COMPILE__
    const double y = __builtin_amdgcn_rsq(v);
    const double h = 0.5 * v * y;
    return y * fma(-h, y, 1.5);
#else
    return 1.0 / sqrt(v);
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

// ------------------------------------------------------------ cubic
// The isolated real root of a monic cubic in closed form (Cardano for one
// real root, the trigonometric form for three), in precision T.  The pencil
// cubic of the intersection below takes its seed from here and refines it
// in FP64.

// Elementary functions for the templated cubic.  FP64: the accurate library
// functions.  FP32 (seeds only, refined in FP64 afterwards): hardware
// approximations -- square root and reciprocal by the single-instruction
// units (about one ulp, no correction sequence), cube root through the base-2
// exponential and logarithm units, arc cosine by the four-term approximation
// of Abramowitz & Stegun 4.4.45 (|error| < 7e-5 rad), cosine through the
// revolution-scaled hardware unit.
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
    const float r = tsqrt(1.0f - ax) * (1.5707288f + ax * (-0.2121144f + ax * (0.0742610f - 0.0187293f * ax)));
    return x < 0.0f ? 3.14159265358979f - r : r;
}
HF_HD __forceinline__ double tcos(double a) { return cos(a); }
HF_HD __forceinline__ float tcos(float a) {
#ifdef __HIP_DEVICE_COMPILE__
    return __builtin_amdgcn_cosf(a * 0.15915494309189535f);  // radians -> revolutions
#else
    return cosf(a);
#endif
}
HF_HD __forceinline__ float tmin(float a, float b) { return fminf(a, b); }
HF_HD __forceinline__ double tmin(double a, double b) { return fmin(a, b); }
HF_HD __forceinline__ float tmax(float a, float b) { return fmaxf(a, b); }
HF_HD __forceinline__ double tmax(double a, double b) { return fmax(a, b); }

// The real root of s^3 + A s^2 + B s + C farthest from the others, in
// precision T: the only real root when there is one; of three, the end root
// on the side of the larger gap.  In the depressed form u^3 + p u + q (roots
// summing to zero) that is the root of largest magnitude, whose sign is that
// of -q: Cardano's real root, or 2 r cos(acos(|c|) / 3) with the sign of c
// for three roots, r = sqrt(-p / 3), c = -q / (2 r^3).
template <typename T>
HF_HD __forceinline__ T cubic_isolated_root(T A, T B, T C) {
    const T third = (T)(1.0 / 3.0);
    const T a3 = A * third;
    const T p = B - A * a3;
    const T q = (T)2 * a3 * a3 * a3 - a3 * B + C;
    const T h = (T)0.5 * q;
    const T p3 = p * third;
    const T disc = h * h + p3 * p3 * p3;
    T u;
    if (disc > (T)0) {
        const T sq = tsqrt(disc);
        const T w = -h - (h >= (T)0 ? sq : -sq);
        const T cu = tcbrt(w);
        u = (cu != (T)0) ? cu - p3 * trcp(cu) : (T)0;
    } else {
        const T rr = tsqrt(tmax(-p3, (T)0));
        T c = (rr > (T)0) ? -h * trcp(rr * rr * rr) : (T)0;
        c = tmin(tmax(c, (T)-1), (T)1);
        const T m = (T)2 * rr * tcos(tacos(c >= (T)0 ? c : -c) * third);
        u = c >= (T)0 ? m : -m;
    }
    return u - a3;
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

// ------------------------------------------------ two-conic intersection
// The real common points of two conics P and Q (section 4: the neutrino's
// transverse momentum satisfies both mass-shell conditions) from their
// pencil.  Written as symmetric 3 x 3 matrices, some member D = A + t B (or
// B + s A) of the pencil is degenerate: det(A + t B) = det A + t tr(adj(A) B)
// + t^2 tr(A adj(B)) + t^3 det B = 0, a cubic.  Its roots are the three ways
// of splitting the four common points into two pairs, D being the pair of
// lines through them.  With four real points, all three splittings are real
// line pairs; with two real and two complex points, only one splitting is
// real (the real chord and the line through the conjugate pair), and the
// cubic has that one real root; with no real point, every splitting gives
// either two real lines that miss the conics or a conjugate pair of lines.
// So one real root suffices: the one farthest from the others (where two
// roots approach each other, two common points do too, and the isolated
// root's lines are the well-conditioned ones).  The adjugate of D is
// -p p^T for the lines' common point p, so a negative diagonal entry means
// a real pair (otherwise there is no real common point); D + [p]_x (the
// cross-product matrix of p) then has rank one, its largest row and column
// being the two lines, and each line meets P in the roots of a quadratic
// along it.  The cubic is taken with its larger end coefficient leading;
// the isolated root comes from the closed form in precision T and is
// refined by two FP64 Newton steps (a seed within 1e-4 relative is then
// correct to rounding).

struct Sym3 {
    double a00, a01, a02, a11, a12, a22;
};

HF_HD __forceinline__ Sym3 sym_adj(const Sym3 &a) {
    return Sym3{a.a11 * a.a22 - a.a12 * a.a12, a.a02 * a.a12 - a.a01 * a.a22, a.a01 * a.a12 - a.a02 * a.a11,
                a.a00 * a.a22 - a.a02 * a.a02, a.a01 * a.a02 - a.a00 * a.a12, a.a00 * a.a11 - a.a01 * a.a01};
}

// tr(X Y) of two symmetric matrices
HF_HD __forceinline__ double sym_trprod(const Sym3 &x, const Sym3 &y) {
    return x.a00 * y.a00 + x.a11 * y.a11 + x.a22 * y.a22 + 2.0 * (x.a01 * y.a01 + x.a02 * y.a02 + x.a12 * y.a12);
}

// The pencil is taken in coordinates u = x / kPencilUnit, where the
// quadratic, linear and constant terms of the mass-shell conics are of one
// size, and each matrix is divided by its largest entry: the cubic's end
// coefficients then compare the conics' degeneracy, not their scales (a side
// whose lepton and b jet are nearly parallel along the beam gives a conic
// many orders of magnitude larger than the other).
constexpr double kPencilUnit = 100.0;

HF_HD __forceinline__ Sym3 sym_balanced(const Conic &q) {
    // kPencilUnit^2, half of it and half of kPencilUnit
    const double s2 = 1e4, s2h = 5e3, s1h = 50.0;
    Sym3 m{q.xx * s2, q.xy * s2h, q.x * s1h, q.yy * s2, q.y * s1h, q.c};
    const double mx = fmax(fmax(fmax(fabs(m.a00), fabs(m.a01)), fmax(fabs(m.a02), fabs(m.a11))),
                           fmax(fabs(m.a12), fabs(m.a22)));
    const double inv = mx > 0.0 ? step_rcp(mx) : 1.0;
    m.a00 *= inv;
    m.a01 *= inv;
    m.a02 *= inv;
    m.a11 *= inv;
    m.a12 *= inv;
    m.a22 *= inv;
    return m;
}

// Common points of line l0 u + l1 v + l2 = 0 and the conic of symmetric
// matrix m: the roots of the conic along the line through its foot point r0
// with direction d = (-l1, l0).
HF_HD __forceinline__ int line_conic(double l0, double l1, double l2, const Sym3 &m, double &xa, double &ya,
                                     double &xb, double &yb) {
    const double n2 = l0 * l0 + l1 * l1;
    if (!(n2 > 0.0)) return 0;
    const double in2 = step_rcp(n2);
    const double x0 = -l2 * l0 * in2, y0 = -l2 * l1 * in2, dx = -l1, dy = l0;
    // half the gradient at r0 and the conic's value there
    const double g0 = fma(m.a00, x0, fma(m.a01, y0, m.a02)), g1 = fma(m.a01, x0, fma(m.a11, y0, m.a12));
    const double c = fma(x0, g0, fma(y0, g1, fma(m.a02, x0, fma(m.a12, y0, m.a22))));
    const double a = fma(dx, fma(m.a00, dx, m.a01 * dy), dy * fma(m.a01, dx, m.a11 * dy));
    const double b = 2.0 * fma(g0, dx, g1 * dy);
    const double disc = fma(b, b, -4.0 * a * c);
    if (!(disc >= 0.0) || a == 0.0) return 0;
    const double sq = fast_sqrt(disc);
    const double t = -0.5 * (b + (b >= 0.0 ? sq : -sq));
    if (t == 0.0) return 0;
    const double s1 = t * step_rcp(a), s2 = c * step_rcp(t);
    xa = fma(s1, dx, x0);
    ya = fma(s1, dy, y0);
    xb = fma(s2, dx, x0);
    yb = fma(s2, dy, y0);
    return 2;
}

struct Points4 {
    double x0, y0, x1, y1, x2, y2, x3, y3;
    int n;
};

// The terms of P that every intersection with it shares: its matrix, the
// adjugate and the determinant.
struct PencilP {
    Sym3 m, adj;
    double det;
};

HF_HD __forceinline__ PencilP pencil_p(const Conic &P) {
    PencilP r;
    r.m = sym_balanced(P);
    r.adj = sym_adj(r.m);
    r.det = r.m.a00 * r.adj.a00 + r.m.a01 * r.adj.a01 + r.m.a02 * r.adj.a02;
    return r;
}

template <typename T>
HF_HD __forceinline__ Points4 conic_intersections(const Conic &P, const PencilP &pp, const Conic &Q) {
    Points4 R;
    R.n = 0;
    R.x0 = R.y0 = R.x1 = R.y1 = R.x2 = R.y2 = R.x3 = R.y3 = 0.0;
    const Sym3 &A = pp.m, &aA = pp.adj;
    const Sym3 B = sym_balanced(Q), aB = sym_adj(B);
    const double dA = pp.det;
    const double dB = B.a00 * aB.a00 + B.a01 * aB.a01 + B.a02 * aB.a02;
    const double c1 = sym_trprod(aA, B), c2 = sym_trprod(A, aB);
    // f(t) = det(U + t W) with |det W| >= |det U|
    const bool swap = fabs(dB) < fabs(dA);
    const double lead = swap ? dA : dB;
    if (!(lead != 0.0) || !isfinite(lead)) return R;
    const double il = fast_rcp(lead);
    const double ca = (swap ? c1 : c2) * il, cb = (swap ? c2 : c1) * il, cc = (swap ? dB : dA) * il;
    double t = (fmax(fabs(ca), fmax(fabs(cb), fabs(cc))) < 1e6)
                   ? (double)cubic_isolated_root<T>((T)ca, (T)cb, (T)cc)
                   : cubic_isolated_root<double>(ca, cb, cc);
    for (int it = 0; it < 2; ++it) {
        const double f = fma(fma(t + ca, t, cb), t, cc), d = fma(fma(3.0, t, 2.0 * ca), t, cb);
        if (d != 0.0) t -= f * step_rcp(d);
    }
    // D = A + t B, or B + t A after the swap (any multiple of it will do)
    const double ta = swap ? t : 1.0, tb = swap ? 1.0 : t;
    const Sym3 D{fma(ta, A.a00, tb * B.a00), fma(ta, A.a01, tb * B.a01), fma(ta, A.a02, tb * B.a02),
                 fma(ta, A.a11, tb * B.a11), fma(ta, A.a12, tb * B.a12), fma(ta, A.a22, tb * B.a22)};
    const Sym3 aD = sym_adj(D);
    // the diagonal entry of largest magnitude; real lines need it < 0
    int ii = 0;
    double bii = aD.a00;
    if (fabs(aD.a11) > fabs(bii)) {
        ii = 1;
        bii = aD.a11;
    }
    if (fabs(aD.a22) > fabs(bii)) {
        ii = 2;
        bii = aD.a22;
    }
    if (!(-bii > 0.0)) return R;
    const double ib = step_rsqrt(-bii);
    const double p0 = (ii == 0 ? aD.a00 : ii == 1 ? aD.a01 : aD.a02) * ib;
    const double p1 = (ii == 0 ? aD.a01 : ii == 1 ? aD.a11 : aD.a12) * ib;
    const double p2 = (ii == 0 ? aD.a02 : ii == 1 ? aD.a12 : aD.a22) * ib;
    // C = D + [p]_x, rank one: the lines are its largest row and column
    const double c00 = D.a00, c01 = D.a01 + p2, c02 = D.a02 - p1;
    const double c10 = D.a01 - p2, c11 = D.a11, c12 = D.a12 + p0;
    const double c20 = D.a02 + p1, c21 = D.a12 - p0, c22 = D.a22;
    // the row holding the entry of largest magnitude, then that entry's column
    const double r0 = fmax(fabs(c00), fmax(fabs(c01), fabs(c02)));
    const double r1 = fmax(fabs(c10), fmax(fabs(c11), fabs(c12)));
    const double r2 = fmax(fabs(c20), fmax(fabs(c21), fabs(c22)));
    const bool row1 = r1 > r0;
    const bool row2 = r2 > (row1 ? r1 : r0);
    const double la0 = row2 ? c20 : row1 ? c10 : c00;
    const double la1 = row2 ? c21 : row1 ? c11 : c01;
    const double la2 = row2 ? c22 : row1 ? c12 : c02;
    const bool col1 = fabs(la1) > fabs(la0);
    const bool col2 = fabs(la2) > (col1 ? fabs(la1) : fabs(la0));
    const double lb0 = col2 ? c02 : col1 ? c01 : c00;
    const double lb1 = col2 ? c12 : col1 ? c11 : c10;
    const double lb2 = col2 ? c22 : col1 ? c21 : c20;
    double xa, ya, xb, yb;
    if (line_conic(la0, la1, la2, A, xa, ya, xb, yb)) {
        R.x0 = xa;
        R.y0 = ya;
        R.x1 = xb;
        R.y1 = yb;
        R.n = 2;
    }
    if (line_conic(lb0, lb1, lb2, A, xa, ya, xb, yb)) {
        if (R.n == 0) {
            R.x0 = xa;
            R.y0 = ya;
            R.x1 = xb;
            R.y1 = yb;
        } else {
            R.x2 = xa;
            R.y2 = ya;
            R.x3 = xb;
            R.y3 = yb;
        }
        R.n += 2;
    }
    R.x0 *= kPencilUnit;
    R.y0 *= kPencilUnit;
    R.x1 *= kPencilUnit;
    R.y1 *= kPencilUnit;
    R.x2 *= kPencilUnit;
    R.y2 *= kPencilUnit;
    R.x3 *= kPencilUnit;
    R.y3 *= kPencilUnit;
    return R;
}

}  // namespace hf
