"""Pins of the oracle's SSP-RK(3,3) (Sec. 3.1, the explicit half of IMEX(3,3,2)).

* Its tableau is the printed one (tests/golden/table_ssprk33.txt), and the
  printed c column equals the row sums of A.
* The tableau satisfies the order conditions up to third order and not the
  fourth-order one sum b A A c = 1/24.
* Stepping y' = lambda y with the oracle's stage combinations converges at third
  order (global error ratio ~8 per halving of dt).
"""
import os
from fractions import Fraction

import numpy as np


def golden():
    path = os.path.join(os.path.dirname(__file__), "golden", "table_ssprk33.txt")
    lines = [l.split("#")[0].split() for l in open(path)]
    lines = [l for l in lines if l]
    c = [Fraction(x) for x in lines[0][1:]]
    A = [[Fraction(x) for x in lines[2 + i]] for i in range(3)]
    b = [Fraction(x) for x in lines[5][1:]]
    assert lines[0][0] == "explicit_c" and lines[1][0] == "explicit_A" and lines[5][0] == "explicit_b"
    return c, A, b


def test_tableau_is_the_printed_one(orc):
    c, A, b = golden()
    Ao, bo = orc.ssprk3_tableau()
    np.testing.assert_array_equal(Ao, np.array([[float(x) for x in r] for r in A]))
    np.testing.assert_allclose(bo, [float(x) for x in b], rtol=0, atol=1e-16)
    assert [sum(r) for r in A] == c


def test_order_conditions():
    c, A, b = golden()
    assert sum(b) == 1
    assert sum(bi * ci for bi, ci in zip(b, c)) == Fraction(1, 2)
    assert sum(bi * ci * ci for bi, ci in zip(b, c)) == Fraction(1, 3)
    assert sum(b[i] * A[i][j] * c[j] for i in range(3) for j in range(3)) == Fraction(1, 6)
    # a fourth-order condition a three-stage explicit method cannot meet
    Ac = [sum(A[i][j] * c[j] for j in range(3)) for i in range(3)]
    assert sum(b[i] * A[i][j] * Ac[j] for i in range(3) for j in range(3)) != Fraction(1, 24)


def test_third_order_convergence_on_linear_decay(orc):
    g = orc.make_grid((4, 1, 1), (1.0, 1.0, 1.0), ng=0)
    lam = np.array([-0.5, -1.0, -2.0, -3.0]).reshape(1, 1, 1, 4)
    errs = []
    for n in (20, 40, 80):
        dt = 1.0 / n
        y = np.ones_like(lam)
        for _ in range(n):
            K, ys = [], y.copy()
            for s in range(3):
                K.append(np.ascontiguousarray(lam * ys))
                nxt = np.zeros_like(y)
                orc.ssprk3_combine(g, 1, s, dt, y, K, nxt)
                ys = nxt
            y = ys
        errs.append(np.abs(y - np.exp(lam)).max())
    r = [np.log2(errs[0] / errs[1]), np.log2(errs[1] / errs[2])]
    assert all(2.8 < x < 3.2 for x in r), r
