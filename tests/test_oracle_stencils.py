"""Pins of the oracle's discrete operators (Sec. 3.2, 3.3).

* the printed coefficients (tests/golden/stencils.txt, Sec. 3.2-3.3) are
  recovered by applying each operator to unit impulses;
* polynomial exactness: centred D1 and both upwind operators exact to degree 4,
  compact D2 to degree 5, KO annihilates degree <= 5, mixed D_xy exact for
  degree <= 4 per axis; each fails one degree higher (so the order is the
  stated one, not an accident of the test data);
* MP5: the conservative difference of unlimited reconstructions is exact for
  polynomials of degree <= 5 on monotone data; constant data -> exact zero;
  no new extrema across a jump.
"""
import ctypes as C
import os
from fractions import Fraction

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden", "stencils.txt")


def golden():
    out = {}
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        parts = line.split()
        den = int(parts[1])
        w = {}
        for t in parts[2:]:
            o, c = t.split(":")
            w[int(o)] = Fraction(int(c), den)
        out[parts[0]] = w
    return out


def _apply(orc, name, u, p, h=1.0):
    L = orc.lib()
    ptr = orc.ptr(u)
    if name == "D1":
        return L.orc_d1(ptr, p, 1, h)
    if name == "D2":
        return L.orc_d2(ptr, p, 1, h)
    if name == "UPW_NEG":
        return L.orc_dup(ptr, p, 1, h, -1.0)
    if name == "UPW_POS":
        return L.orc_dup(ptr, p, 1, h, 1.0)
    if name == "KO":
        return L.orc_ko(ptr, p, 1, h, 1.0)
    raise KeyError(name)


@pytest.mark.parametrize("name", ["D1", "D2", "UPW_NEG", "UPW_POS", "KO"])
def test_printed_coefficients(orc, name):
    w = golden()[name]
    n = 9
    for off in range(-3, 4):
        u = np.zeros(n)
        u[4 + off] = 1.0
        got = _apply(orc, name, u, 4)
        want = float(w.get(off, Fraction(0)))
        assert got == pytest.approx(want, abs=1e-15), (name, off)


def test_mp5_printed_unlimited_weights(orc):
    # the unlimited interpolant is the reconstruction on monotone data; weights
    # recovered by finite differences around a monotone base profile
    w = golden()["MP5"]
    base = np.array([0.0, 1.0, 2.0, 3.0, 4.0])
    f0 = orc.mp5(base)
    for m in range(5):
        e = 1e-6
        b = base.copy()
        b[m] += e
        assert (orc.mp5(b) - f0) / e == pytest.approx(float(w[m - 2]), rel=1e-6)


def _poly(coefs, x):
    return sum(float(c) * x ** k for k, c in enumerate(coefs))


def _exact_deriv(coefs, x, order):
    s = Fraction(0)
    for k, c in enumerate(coefs):
        if k >= order:
            f = Fraction(1)
            for t in range(order):
                f *= k - t
            s += c * f * Fraction(x) ** (k - order)
    return s


RNG = np.random.default_rng(7)


def rand_coefs(deg):
    return [Fraction(int(RNG.integers(-5, 6))) for _ in range(deg)] + [Fraction(int(RNG.choice([-3, -2, -1, 1, 2, 3])))]


@pytest.mark.parametrize("name,order,exact_deg", [("D1", 1, 4), ("UPW_NEG", 1, 4), ("UPW_POS", 1, 4),
                                                  ("D2", 2, 5)])
def test_polynomial_exactness(orc, name, order, exact_deg):
    h = Fraction(1, 8)
    xc = Fraction(3, 8)
    for deg in range(0, exact_deg + 2):
        for _ in range(3):
            co = rand_coefs(deg)
            xs = [xc + m * h for m in range(-4, 5)]
            u = np.array([_poly(co, float(x)) for x in xs])
            got = _apply(orc, name, u, 4, float(h))
            want = float(_exact_deriv(co, xc, order))
            scale = max(1.0, max(abs(float(c)) for c in co)) * 50
            if deg <= exact_deg:
                assert abs(got - want) <= 1e-12 * scale, (name, deg)
            else:
                assert abs(got - want) > 1e-9, (name, deg)


def test_ko_annihilates_degree5(orc):
    h = Fraction(1, 4)
    for deg in range(0, 7):
        co = rand_coefs(deg)
        xs = [m * h for m in range(-4, 5)]
        u = np.array([_poly(co, float(x)) for x in xs])
        got = _apply(orc, "KO", u, 4, float(h))
        if deg <= 5:
            assert abs(got) < 1e-11
        else:
            # sigma/(64h) * h^6 * 6! * c6
            want = 1.0 / 64.0 * float(h) ** 5 * 720 * float(co[6])
            assert got == pytest.approx(want, rel=1e-9)


def test_mixed_derivative_exact(orc):
    hx, hy = 0.125, 0.25
    nx, ny = 9, 9
    X, Y = np.meshgrid((np.arange(nx) - 4) * hx, (np.arange(ny) - 4) * hy, indexing="xy")
    # u = sum a_jk x^j y^k with j,k <= 4 ; d2u/dxdy exact
    a = RNG.integers(-3, 4, size=(5, 5)).astype(float)
    u = sum(a[j, k] * X ** j * Y ** k for j in range(5) for k in range(5))
    want = a[1, 1]   # value at the origin
    arr = np.ascontiguousarray(u)
    p = 4 + nx * 4
    got = orc.lib().orc_d11(orc.ptr(arr), p, 1, nx, hx, hy)
    assert got == pytest.approx(want, abs=1e-10)
    # degree 5 in x breaks it
    u2 = u + X ** 5 * Y
    got2 = orc.lib().orc_d11(orc.ptr(np.ascontiguousarray(u2)), p, 1, nx, hx, hy)
    assert abs(got2 - want) > 1e-6


def test_mp5_conservative_difference_exact(orc):
    """(Fhat_{i+1/2} - Fhat_{i-1/2})/h = F'(x_i) for monotone polynomials of degree <= 5."""
    h = 0.05
    for deg in range(1, 7):
        # monotone increasing on the stencil: F = x + c x^deg with small c
        c = 0.3
        xs = (np.arange(-3, 4)) * h + 0.2
        F = xs + c * xs ** deg
        fr = orc.mp5(F[1:6])    # interface i+1/2 from i-2..i+2
        fl = orc.mp5(F[0:5])    # interface i-1/2
        got = (fr - fl) / h
        want = 1.0 + c * deg * 0.2 ** (deg - 1)
        if deg <= 5:
            assert got == pytest.approx(want, rel=1e-11, abs=1e-11), deg
        else:
            assert abs(got - want) > 1e-12, deg


def test_mp5_constant_and_jump(orc):
    assert orc.mp5([0.7] * 5) == 0.7 or abs(orc.mp5([0.7] * 5) - 0.7) < 1e-16
    # a step: the reconstruction stays within the neighbouring values
    for f5 in ([0, 0, 0, 1, 1], [0, 0, 1, 1, 1], [1, 1, 1, 0, 0], [0, 0, 0, 0, 1], [0, 1, 1, 1, 1]):
        v = orc.mp5(np.array(f5, dtype=float))
        assert min(f5[2], f5[3]) - 1e-15 <= v <= max(f5[2], f5[3]) + 1e-15, f5


def test_mp5_smooth_extremum_not_clipped(orc):
    """Near a smooth extremum the limiter keeps the unlimited interpolant
    (weights printed in Sec. 3.3, tests/golden/stencils.txt) once h is small."""
    w = golden()["MP5"]
    for h in (0.02, 0.01):
        for x0 in np.linspace(-3 * h, 3 * h, 13):
            f5 = np.cos(x0 + h * np.arange(-2, 3))
            unl = sum(float(w[m - 2]) * f5[m] for m in range(5))
            got = orc.mp5(f5)
            assert got == pytest.approx(unl, rel=1e-13, abs=1e-15), (h, x0)


# Limited MP5 values worked by hand from the bounds of Sec. 3.3 (alpha = 4).
# F = (F_{i-2}, F_{i-1}, F_i, F_{i+1}, F_{i+2}); D+ = F_{i+1} - F_i, D- = F_i - F_{i-1};
# d_{i-1}, d_i, d_{i+1} are the second differences centred on i-1, i, i+1.
MP5_LIMITED = [
    # (-4, 3, 6, 6, -5): unlimited 412/60 = 103/15; f^MP = 6 + minmod(0, 12) = 6, so the
    # test (103/15 - 6)^2 < 0 fails and the limiter acts.  d = (-4, -3, -11):
    # d^M4_{i+1/2} = minmod(-12+11, -44+3, -3, -11) = -1, d^M4_{i-1/2} = minmod(-16+3, -12+4, -4, -3) = -3.
    # f^UL = 6 + 12 = 18, f^MD = 6 + 1/2 = 13/2, f^LC = 6 + 3/2 + (4/3)(-3) = 7/2.
    # f^min = max(min(6, 6, 13/2), min(6, 18, 7/2)) = 6, f^max = min(13/2, 18) = 13/2:
    # the result is f^MD.
    ((-4, 3, 6, 6, -5), Fraction(13, 2)),
    # (1, -3, -5, 0, 3): unlimited -203/60; f^MP = -5 + minmod(5, -8) = -5, limiter acts.
    # d = (2, 7, -2): d^M4_{i+1/2} = minmod(30, -15, 7, -2) = 0 (mixed signs),
    # d^M4_{i-1/2} = minmod(1, 26, 2, 7) = 1.  f^UL = -13, f^MD = -5/2, f^LC = -5 - 1 + 4/3 = -14/3.
    # f^min = max(-5, -13) = -5, f^max = min(max(-5, 0, -5/2), max(-5, -13, -14/3)) = -14/3:
    # the result is f^LC, through the 4/3 curvature term.
    ((1, -3, -5, 0, 3), Fraction(-14, 3)),
    # (6, 6, 5, -5, -2): unlimited 40/60 = 2/3; f^MP = 5 + minmod(-10, -4) = 1 and
    # (2/3 - 5)(2/3 - 1) > 0, limiter acts.  d = (-1, -9, 13): both d^M4 are 0 (mixed signs).
    # f^UL = 5 - 4 = 1, f^MD = 0, f^LC = 9/2; f^min = max(-5, 1) = 1, f^max = min(5, 5) = 5:
    # the result is f^UL.
    ((6, 6, 5, -5, -2), Fraction(1)),
    # (-5, 1, 4, -2, -6): unlimited 129/60 = 43/20; f^MP = 4 + minmod(-6, 12) = 4, limiter acts.
    # d = (-3, -9, 2): d^M4_{i+1/2} = 0, d^M4_{i-1/2} = minmod(-3, -33, -3, -9) = -3.
    # f^UL = 16, f^MD = 1, f^LC = 4 + 3/2 - 4 = 3/2; f^min = max(-2, 3/2) = 3/2, f^max = min(4, 16) = 4:
    # 43/20 lies inside [3/2, 4] and is kept (a wrong f^LC above 43/20 would move it).
    ((-5, 1, 4, -2, -6), Fraction(43, 20)),
]


def check_mp5_limited(orc):
    for f5, want in MP5_LIMITED:
        got = orc.mp5(np.array(f5, dtype=float))
        assert got == pytest.approx(float(want), rel=2e-16, abs=0), (f5, got, want)
        # mirrored data (the right-state reconstruction reads the stencil reversed and
        # negated values flip every bound): R(-F) = -R(F)
        got_neg = orc.mp5(-np.array(f5, dtype=float))
        assert got_neg == pytest.approx(-float(want), rel=2e-16, abs=0), (f5, got_neg)


def test_mp5_limited_values(orc):
    check_mp5_limited(orc)
