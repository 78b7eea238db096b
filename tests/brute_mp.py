"""50-digit brute-force solution of the two-neutrino system for one pairing.

An independent route to the same answer as the oracle, used only by tests:
  * (E, p_z) of each neutrino come from a 2x2 linear solve (mpmath LU) of the
    W- and top-mass conditions at each sampled (x, y);
  * the two mass-shell conics are only ever *evaluated*;
  * the eliminant in y is the 4x4 Sylvester determinant of the two quadratics
    in y, evaluated numerically at seven x points and interpolated (degree at
    most four, checked);
  * all complex roots come from mpmath.polyroots;
  * y is the common root of the two quadratics in y.
"""

import mpmath as mp

mp.mp.dps = 50

XS = mp.mpf(100)


def _m(v):
    return [mp.mpf(float(a)) for a in v]


def _dot(a, b):
    return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3]


class _Side:
    def __init__(self, lep, b, mt, mw):
        self.l, self.b = lep, b
        mt, mw = mp.mpf(float(mt)), mp.mpf(float(mw))
        self.kl = (mw ** 2 - _dot(lep, lep)) / 2
        self.kb = (mt ** 2 - mw ** 2 - _dot(b, b) - 2 * _dot(b, lep)) / 2
        self.M = mp.matrix([[lep[0], -lep[3]], [b[0], -b[3]]])

    def ez(self, x, y):
        r = mp.matrix([self.kl + self.l[1] * x + self.l[2] * y, self.kb + self.b[1] * x + self.b[2] * y])
        s = mp.lu_solve(self.M, r)
        return s[0], s[1]

    def shell(self, x, y):
        e, z = self.ez(x, y)
        return e * e - x * x - y * y - z * z


def _quad_in_y(f):
    """Coefficients (a, b, c) of the quadratic y -> f(y) from three samples."""
    f0, f1, fm = f(mp.mpf(0)), f(mp.mpf(1)), f(mp.mpf(-1))
    return (f1 + fm) / 2 - f0, (f1 - fm) / 2, f0


def solve(lp, b, lm, bb, metx, mety, mt=172.5, mw=80.4):
    """Accepted solutions [(x, y, z, E, xb, yb, zb, Eb)] as mpf, ascending in x,
    plus the minimum separation of the real roots of the eliminant."""
    s1 = _Side(_m(lp), _m(b), mt, mw)
    s2 = _Side(_m(lm), _m(bb), mt, mw)
    mx, my = mp.mpf(float(metx)), mp.mpf(float(mety))

    def pq(x):
        P = _quad_in_y(lambda y: s1.shell(x, y))
        Q = _quad_in_y(lambda y: s2.shell(mx - x, my - y))
        return P, Q

    def eliminant(x):
        (a, b_, c), (d, e, f) = pq(x)
        S = mp.matrix([[a, b_, c, 0], [0, a, b_, c], [d, e, f, 0], [0, d, e, f]])
        return mp.det(S)

    ts = [mp.mpf(k) for k in (-3, -2, -1, 0, 1, 2, 3)]
    vals = [eliminant(XS * t) for t in ts]
    V = mp.matrix([[t ** k for k in range(5)] for t in ts[:5]])
    coef = mp.lu_solve(V, mp.matrix(vals[:5]))
    scale = max(abs(c) for c in coef)
    for t, v in zip(ts[5:], vals[5:]):
        pred = sum(coef[k] * t ** k for k in range(5))
        assert abs(pred - v) <= mp.mpf(10) ** -35 * scale * 7 ** 4, "eliminant is not a quartic"
    cs = [coef[k] for k in range(5)]
    while len(cs) > 1 and abs(cs[-1]) <= mp.mpf(10) ** -40 * scale:
        cs.pop()
    if len(cs) <= 1:
        return [], mp.inf
    roots = mp.polyroots(cs[::-1], maxsteps=400, extraprec=200)
    real = sorted(XS * mp.re(r) for r in roots if abs(mp.im(r)) <= mp.mpf(10) ** -30 * max(1, abs(r)))
    sep = min([abs(real[i + 1] - real[i]) for i in range(len(real) - 1)] + [mp.inf])
    out = []
    for x in real:
        (a, b_, c), (d, e, f) = pq(x)
        ys = []
        if a != 0:
            disc = b_ * b_ - 4 * a * c
            sq = mp.sqrt(disc) if disc >= 0 else None
            if sq is not None:
                ys = [(-b_ - sq) / (2 * a), (-b_ + sq) / (2 * a)]
        elif b_ != 0:
            ys = [-c / b_]
        if not ys:
            continue
        y = min(ys, key=lambda yy: abs(d * yy * yy + e * yy + f))
        en, zn = s1.ez(x, y)
        xb, yb = mx - x, my - y
        eb, zb = s2.ez(xb, yb)
        if en < 0 or eb < 0:
            continue
        out.append((x, y, zn, en, xb, yb, zb, eb))
    return out, sep
