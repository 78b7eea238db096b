// Algorithmic floating-point operation count of the reconstruction search,
// per unit of work, obtained by running the search kernel's own math
// (hf_reco_math.hpp) on the host with counting scalar types.
//
// Counted as one operation each: add/sub, mul, div (also the reciprocal
// estimate), sqrt, transcendental; FMA as two.  Comparisons, selections and
// integer work (the counter-based generator) are not counted.  FP64 and FP32
// operations are tallied separately.
//
// Input (binary, float64 rows of 18 values): l+ (E, px, py, pz), b, l-,
// bbar, MET x, MET y, of one smeared pairing.  Output: the mean operation
// counts per pairing (the l- side's varying terms, the reflection through
// the MET, the pencil cubic, its line pair and the two line-conic
// quadratics) and per intersection point (polish, acceptance, energies'
// signs, score), and the number of pairings and points.
#include <cmath>
#include <cstdio>
#include <vector>

#include <hip/hip_runtime.h>

struct Tally {
    long add = 0, mul = 0, fma = 0, div = 0, sqrt = 0, trans = 0;
    double flops() const { return (double)add + mul + 2.0 * fma + div + sqrt + trans; }
    void clear() { *this = Tally(); }
};
static Tally T64, T32;

struct CD {  // counting double
    double v;
    constexpr CD() : v(0) {}
    constexpr CD(double x) : v(x) {}
    explicit operator double() const { return v; }
    explicit operator float() const { return (float)v; }
};
struct CF {  // counting float
    float v;
    constexpr CF() : v(0) {}
    constexpr CF(float x) : v(x) {}
    constexpr CF(double x) : v((float)x) {}
    constexpr CF(int x) : v((float)x) {}
    explicit CF(CD x) : v((float)x.v) {}
    explicit operator double() const { return v; }
    explicit operator CD() const { return CD((double)v); }
};

#define BIN(Ty, TA, op, fld)                                                          \
    inline Ty operator op(Ty a, Ty b) { ++TA.fld; return Ty(a.v op b.v); }            \
    inline Ty operator op(Ty a, double b) { ++TA.fld; return Ty(a.v op b); }          \
    inline Ty operator op(double a, Ty b) { ++TA.fld; return Ty(a op b.v); }          \
    inline Ty &operator op##=(Ty &a, Ty b) { ++TA.fld; a.v = a.v op b.v; return a; }  \
    inline Ty &operator op##=(Ty &a, double b) { ++TA.fld; a.v = a.v op b; return a; }
BIN(CD, T64, +, add) BIN(CD, T64, -, add) BIN(CD, T64, *, mul) BIN(CD, T64, /, div)
BIN(CF, T32, +, add) BIN(CF, T32, -, add) BIN(CF, T32, *, mul) BIN(CF, T32, /, div)
inline CD operator-(CD a) { return CD(-a.v); }
inline CF operator-(CF a) { return CF(-a.v); }
#define CMP(Ty, op)                                                   \
    inline bool operator op(Ty a, Ty b) { return a.v op b.v; }        \
    inline bool operator op(Ty a, double b) { return a.v op b; }      \
    inline bool operator op(double a, Ty b) { return a op b.v; }
CMP(CD, <) CMP(CD, >) CMP(CD, <=) CMP(CD, >=) CMP(CD, ==) CMP(CD, !=)
CMP(CF, <) CMP(CF, >) CMP(CF, <=) CMP(CF, >=) CMP(CF, ==) CMP(CF, !=)

inline CD fma(CD a, CD b, CD c) { ++T64.fma; return CD(std::fma(a.v, b.v, c.v)); }
inline CD fabs(CD a) { return CD(std::fabs(a.v)); }
inline CD fmax(CD a, CD b) { return CD(std::fmax(a.v, b.v)); }
inline CD fmin(CD a, CD b) { return CD(std::fmin(a.v, b.v)); }
inline CD sqrt(CD a) { ++T64.sqrt; return CD(std::sqrt(a.v)); }
inline CD cbrt(CD a) { ++T64.trans; return CD(std::cbrt(a.v)); }
inline CD acos(CD a) { ++T64.trans; return CD(std::acos(a.v)); }
inline CD sin(CD a) { ++T64.trans; return CD(std::sin(a.v)); }
inline CD cos(CD a) { ++T64.trans; return CD(std::cos(a.v)); }
inline bool isfinite(CD a) { return std::isfinite(a.v); }
inline CF fabsf(CF a) { return CF(std::fabs(a.v)); }
inline CF sqrtf(CF a) { ++T32.sqrt; return CF(std::sqrt(a.v)); }
inline CF exp2f(CF a) { ++T32.trans; return CF(std::exp2(a.v)); }
inline CF log2f(CF a) { ++T32.trans; return CF(std::log2(a.v)); }
inline CF sinf(CF a) { ++T32.trans; return CF(std::sin(a.v)); }
inline CF cosf(CF a) { ++T32.trans; return CF(std::cos(a.v)); }
inline CF fminf(CF a, CF b) { return CF(std::fmin(a.v, b.v)); }
inline CF fmaxf(CF a, CF b) { return CF(std::fmax(a.v, b.v)); }
inline CF copysignf(CF a, CF b) { return CF(std::copysign(a.v, b.v)); }

// The math header, with its FP64 type and its FP32 seed type replaced by the
// counting types.
#define double CD
#define float CF
#include "../csrc/hf_reco_math.hpp"
#undef double
#undef float

using namespace hf;

int main(int argc, char **argv) {
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 1;
    std::vector<double> a;
    double buf[18];
    while (fread(buf, 8, 18, f) == 18) a.insert(a.end(), buf, buf + 18);
    const size_t n = a.size() / 18;
    const double mt = 172.5, mw = 80.4;
    Tally s1_64, s1_32, it_64, it_32;
    long pairs = 0, items = 0, accepted = 0;
    auto add = [](Tally &d, const Tally &t) {
        d.add += t.add; d.mul += t.mul; d.fma += t.fma; d.div += t.div; d.sqrt += t.sqrt; d.trans += t.trans;
    };
    for (size_t k = 0; k < n; ++k) {
        const double *r = &a[18 * k];
        CD lp[4] = {r[0], r[1], r[2], r[3]}, b[4] = {r[4], r[5], r[6], r[7]};
        CD lm[4] = {r[8], r[9], r[10], r[11]}, bb[4] = {r[12], r[13], r[14], r[15]};
        CD sp[kSide], sm[kSide];
        // side constants are staged once per event and candidate, and the
        // l+ side's varying terms once per variation and candidate (counted
        // per variation): neither is per pairing
        if (!make_side(lp, b, sp) || !make_side(lm, bb, sm)) continue;
        const CD mt2_mw2 = CD(mt) * CD(mt) - CD(mw) * CD(mw), mw2 = CD(mw) * CD(mw);
        const CD ml2p = lp[0] * lp[0] - lp[1] * lp[1] - lp[2] * lp[2] - lp[3] * lp[3];
        const CD ml2m = lm[0] * lm[0] - lm[1] * lm[1] - lm[2] * lm[2] - lm[3] * lm[3];
        const CD one(1.0);
        const CD Wp = mw2 / (2.0 * one) - 0.5 * one * ml2p, Wm = mw2 / (2.0 * one) - 0.5 * one * ml2m;
        SideVar A = side_var(sp, Wp, one, one, mt2_mw2);
        const PencilP pa = pencil_p(A.q);
        T64.clear();
        T32.clear();
        SideVar B = side_var(sm, Wm, one, one, mt2_mw2);
        Conic Q = reflect(B.q, CD(r[16]), CD(r[17]));
        const Points4 pts = conic_intersections<CF>(A.q, pa, Q);
        add(s1_64, T64);
        add(s1_32, T32);
        ++pairs;
        for (int kk = 0; kk < pts.n; ++kk) {
            T64.clear();
            T32.clear();
            CD x = kk == 0 ? pts.x0 : kk == 1 ? pts.x1 : kk == 2 ? pts.x2 : pts.x3;
            CD y = kk == 0 ? pts.y0 : kk == 1 ? pts.y1 : kk == 2 ? pts.y2 : pts.y3;
            ++items;
            if (polish_xy(A.q, Q, x, y, 4, kPolishSkip * kAcceptM2 * 80.4 * 80.4) <= kAcceptM2 * 80.4 * 80.4) {
                const CD en = sp[kE1] * x + sp[kE2] * y + A.e0;
                const CD xb = CD(r[16]) - x, yb = CD(r[17]) - y;
                const CD eb = sm[kE1] * xb + sm[kE2] * yb + B.e0;
                if (en >= 0.0 && eb >= 0.0) {
                    ++accepted;
                    // score: top pT terms (the point-independent parts are per pairing)
                    const CD tx = one * b[1] + one * lp[1] + x, ty = one * b[2] + one * lp[2] + y;
                    const CD tbx = one * bb[1] + one * lm[1] + xb, tby = one * bb[2] + one * lm[2] + yb;
                    const CD w = -0.5 * one - (sqrt(tx * tx + ty * ty) + sqrt(tbx * tbx + tby * tby)) * CD(0.01);
                    (void)w;
                }
            }
            add(it_64, T64);
            add(it_32, T32);
        }
    }
    auto pr = [](const char *name, const Tally &t, long d) {
        printf("%s add %.2f mul %.2f fma %.2f div %.2f sqrt %.2f trans %.2f flops %.2f\n", name, (double)t.add / d,
               (double)t.mul / d, (double)t.fma / d, (double)t.div / d, (double)t.sqrt / d, (double)t.trans / d,
               t.flops() / d);
    };
    printf("pairings %ld points %ld accepted %ld\n", pairs, items, accepted);
    pr("pairing_fp64_per_pairing", s1_64, pairs);
    pr("pairing_fp32_per_pairing", s1_32, pairs);
    pr("point_fp64_per_point", it_64, items ? items : 1);
    pr("point_fp32_per_point", it_32, items ? items : 1);
    return 0;
}
