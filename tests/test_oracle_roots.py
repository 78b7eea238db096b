"""Pins of the oracle's polynomial real-root step.

Quartics are built from chosen real roots and complex pairs, so the expected
sign-changing real roots are known by construction; numpy.roots serves as a
second library reference on the same polynomials.
"""

import numpy as np
import pytest


def _poly_from_roots(real, cplx=(), lead=1.0):
    r = list(real)
    for c in cplx:
        r += [c, np.conj(c)]
    return np.real(np.poly(r))[::-1] * lead  # ascending coefficients


@pytest.mark.parametrize("seed", range(40))
def test_quartic_roots_match_construction(orc, seed):
    rng = np.random.default_rng(seed)
    kind = seed % 3
    if kind == 0:
        real = np.sort(rng.uniform(-3, 3, 4))
        cplx = ()
    elif kind == 1:
        real = np.sort(rng.uniform(-3, 3, 2))
        cplx = (complex(rng.uniform(-3, 3), rng.uniform(0.05, 2)),)
    else:
        real = np.array([])
        cplx = (complex(rng.uniform(-3, 3), rng.uniform(0.05, 2)),
                complex(rng.uniform(-3, 3), rng.uniform(0.05, 2)))
    lead = rng.choice([-1.0, 1.0]) * 10 ** rng.uniform(-3, 3)
    c = _poly_from_roots(real, cplx, lead)
    got = orc.real_roots(c)
    assert got.size == real.size
    if real.size:
        sep = np.min(np.diff(np.concatenate([[-1e9], real, [1e9]])))
        tol = 1e-12 * max(1.0, 1.0 / sep)
        np.testing.assert_allclose(got, real, rtol=0, atol=tol)
        nr = np.sort(np.real(np.roots(c[::-1])[np.abs(np.imag(np.roots(c[::-1]))) < 1e-9]))
        np.testing.assert_allclose(got, nr, atol=1e-8)


def test_roots_ascending_and_within_bisection_precision(orc):
    c = _poly_from_roots([-2.5, -0.125, 0.75, 1.5])
    got = orc.real_roots(c)
    assert np.all(np.diff(got) > 0)
    for r, w in zip(got, [-2.5, -0.125, 0.75, 1.5]):
        assert abs(r - w) <= 8 * np.spacing(abs(w))


def test_touching_root_not_reported(orc):
    # ((t-1)^2 + 1e-6)(t+2)(t-3): q touches near t=1 without crossing zero
    touch = np.polymul([1.0, -2.0, 1.0 + 1e-6], [1.0, -1.0, -6.0])[::-1]
    np.testing.assert_allclose(orc.real_roots(touch), [-2.0, 3.0], atol=1e-12)
    # ((t-1)^2 - 1e-6)(t+2)(t-3): two crossings 1 -+ 1e-3
    cross = np.polymul([1.0, -2.0, 1.0 - 1e-6], [1.0, -1.0, -6.0])[::-1]
    np.testing.assert_allclose(orc.real_roots(cross), [-2.0, 1 - 1e-3, 1 + 1e-3, 3.0], atol=1e-10)
    # (t-1)^2 (t^2+1) + 1e-9: no sign change at all
    c = _poly_from_roots([1.0, 1.0], (1j,))
    c[0] += 1e-9
    assert orc.real_roots(c).size == 0


def test_exact_double_root_is_numerically_double(orc):
    # an exact double root sits at the rounding limit: reported as nothing or as
    # a pair within sqrt(eps) of it, never as a lone root
    got = orc.real_roots(_poly_from_roots([1.0, 1.0, -2.0, 3.0]))
    near = got[np.abs(got - 1.0) < 1e-3]
    assert near.size in (0, 2)
    assert np.all(np.abs(near - 1.0) < 1e-6)


def test_triple_root_reported_once(orc):
    # (t-0.5)^3 (t+1): odd multiplicity changes sign
    got = orc.real_roots(_poly_from_roots([0.5, 0.5, 0.5, -1.0]))
    assert got.size == 2
    np.testing.assert_allclose(got, [-1.0, 0.5], atol=1e-5)


def test_degree_reduction(orc):
    # leading coefficient below 1e-14 of the largest: treated as a cubic
    c = _poly_from_roots([-1.0, 0.5, 2.0])  # cubic, ascending, len 4
    c5 = np.concatenate([c, [1e-16]])
    np.testing.assert_allclose(orc.real_roots(c5), [-1.0, 0.5, 2.0], atol=1e-12)
    # linear and quadratic special cases
    np.testing.assert_allclose(orc.real_roots([3.0, -2.0]), [1.5])
    np.testing.assert_allclose(orc.real_roots([-4.0, 0.0, 1.0]), [-2.0, 2.0])
    assert orc.real_roots([4.0, 0.0, 1.0]).size == 0
    assert orc.real_roots([0.0, 0.0, 0.0, 0.0, 0.0]).size == 0
    assert orc.real_roots([5.0]).size == 0


def test_wide_dynamic_range(orc):
    # roots spanning six decades
    real = [-1e3, -1.0, 1e-3, 10.0]
    got = orc.real_roots(_poly_from_roots(real))
    np.testing.assert_allclose(got, real, rtol=1e-9)
