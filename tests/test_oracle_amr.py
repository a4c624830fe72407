"""Pins of the oracle's mesh-refinement glue (prolongation, restriction, RK4
dense output) against what the paper prints and what the mathematics fixes.

* The six-point weights computed from the Lagrange basis equal the simplified
  weights printed in Sec. 4.2 (tests/golden/refinement_rk4_dense.txt).
* Prolongation reproduces every polynomial of degree <= 5 in each variable
  (tensor product of the symmetric six-point interpolation) and copies
  coincident points; degree 6 is not reproduced (so the stencil is the
  six-point one, not wider).
* Restriction by copy undoes prolongation at coincident points, bit for bit.
* Dense-output weights equal the printed polynomials, reduce to the RK4
  weights at theta = 1 and to 0 at theta = 0, their theta-derivatives match
  finite differences, and the interpolant is third order for y' = lambda y
  (global error ~ h^4 at fixed theta; first derivative ~ h^3).
"""
import os
from fractions import Fraction

import numpy as np
import pytest

pytestmark = pytest.mark.filterwarnings("ignore")


def golden():
    path = os.path.join(os.path.dirname(__file__), "golden", "refinement_rk4_dense.txt")
    out = {}
    for line in open(path):
        line = line.split("#")[0].split()
        if not line:
            continue
        out[line[0]] = line[1:]
    return out


def grid(orc, n, ng):
    return orc.make_grid(n, (1.0, 1.0, 1.0), ng=ng)


def test_lagrange_weights_are_the_printed_ones(orc):
    g = golden()["PROLONG"]
    den = float(g[0])
    printed = np.array([float(t.split(":")[1]) for t in g[1:]]) / den
    assert [int(t.split(":")[0]) for t in g[1:]] == [-2, -1, 0, 1, 2, 3]
    np.testing.assert_allclose(orc.lagrange_half(), printed, rtol=0, atol=1e-16)


def _poly(x, y, z, cx, cy, cz):
    return np.polynomial.polynomial.polyval(x, cx) * np.polynomial.polynomial.polyval(y, cy) * \
        np.polynomial.polynomial.polyval(z, cz)


def _coarse_fine(orc, deg, seed, nfields=2):
    """Coarse 12^3 + 3 ghosts (x = i), fine 14x12x10 + 3 ghosts placed so that
    fine index I sits at coarse position (I - off)/2, every stencil inside the
    coarse grid, with both parities of the offset; fields are polynomials."""
    r = np.random.default_rng(seed)
    gc, gf = grid(orc, (12, 12, 12), 3), grid(orc, (14, 12, 10), 3)
    Nc = (18, 18, 18)
    Nf = (16, 18, 20)  # z, y, x padded extents of the fine grid
    off = (-6, -7, -5)
    zc, yc, xc = np.meshgrid(*[np.arange(n, dtype=float) for n in Nc], indexing="ij")
    zf, yf, xf = np.meshgrid(*[(np.arange(n) - o) / 2.0 for n, o in zip(Nf, off[::-1])], indexing="ij")
    Uc = np.zeros((nfields,) + Nc)
    Uexact = np.zeros((nfields,) + Nf)
    for f in range(nfields):
        cs = [r.normal(size=d + 1) * 0.3 ** np.arange(d + 1) for d in deg]
        Uc[f] = _poly(xc, yc, zc, *cs)
        Uexact[f] = _poly(xf, yf, zf, *cs)
    return gc, gf, Uc, Uexact, off


@pytest.mark.parametrize("seed", [1, 2])
def test_prolongation_reproduces_degree_five(orc, seed):
    gc, gf, Uc, Ue, off = _coarse_fine(orc, (5, 5, 5), seed)
    Uf = np.full_like(Ue, np.nan)
    lo, hi = (0, 0, 0), (20, 18, 16)  # the whole padded fine grid (x, y, z)
    assert orc.prolong(gc, Uc, gf, Uf, 2, off, lo, hi) == 0
    assert np.isfinite(Uf).all()
    scale = np.abs(Ue).max()
    assert np.abs(Uf - Ue).max() <= 1e-12 * scale
    # coincident points are copies, bit for bit
    zi, yi, xi = [np.arange((o % 2), n, 2) for n, o in zip(Uf.shape[1:], off[::-1])]
    sub = Uf[:, zi][:, :, yi][:, :, :, xi]
    ci = [(np.arange((o % 2), n, 2) - o) // 2 for n, o in zip(Uf.shape[1:], off[::-1])]
    ref = Uc[:, ci[0]][:, :, ci[1]][:, :, :, ci[2]]
    assert np.array_equal(sub, ref)


def test_prolongation_does_not_reproduce_degree_six(orc):
    gc, gf, Uc, Ue, off = _coarse_fine(orc, (6, 0, 0), 3, nfields=1)
    Uf = np.zeros_like(Ue)
    assert orc.prolong(gc, Uc, gf, Uf, 1, off, (0, 0, 0), (20, 18, 16)) == 0
    assert np.abs(Uf - Ue).max() > 1e-9 * np.abs(Ue).max()  # degree 5 reaches 1e-12


def test_prolongation_rejects_points_without_coarse_support(orc):
    gc, gf, Uc, Ue, off = _coarse_fine(orc, (1, 1, 1), 4, nfields=1)
    Uf = np.zeros_like(Ue)
    # a fine x index whose six-point stencil runs past the coarse grid
    bad_off = (-1, -7, -5)
    assert orc.prolong(gc, Uc, gf, Uf, 1, bad_off, (0, 0, 0), (20, 18, 16)) == -1


def test_restriction_undoes_prolongation(orc):
    gc, gf, Uc, Ue, off = _coarse_fine(orc, (5, 4, 3), 5)
    Uf = np.zeros_like(Ue)
    assert orc.prolong(gc, Uc, gf, Uf, 2, off, (0, 0, 0), (20, 18, 16)) == 0
    back = np.full_like(Uc, -7.0)
    # coarse points covered by the fine grid: I = 2 i + off within [0, N_f)
    lo = [max(0, (1 - o) // 2) for o in off]
    hi = [min(18, (n - 1 - o) // 2 + 1) for n, o in zip((20, 18, 16), off)]
    assert orc.restrict(gf, Uf, gc, back, 2, off, lo, hi) == 0
    sl = (slice(None), slice(lo[2], hi[2]), slice(lo[1], hi[1]), slice(lo[0], hi[0]))
    assert np.array_equal(back[sl], Uc[sl])
    mask = np.ones(back.shape, bool)
    mask[sl] = False
    assert (back[mask] == -7.0).all()
    assert orc.restrict(gf, Uf, gc, back, 2, off, lo, [h + 1 for h in hi]) == -1


def _printed_b(theta):
    g = golden()
    out = []
    for name in ("B1", "B2", "B3", "B4"):
        c = [Fraction(t) for t in g[name]]
        out.append(float(sum(ci * Fraction(theta) ** (p + 1) for p, ci in enumerate(c))))
    return np.array(out)


@pytest.mark.parametrize("theta", [0.0, 0.25, 0.5, 0.8, 1.0])
def test_dense_weights_are_the_printed_polynomials(orc, theta):
    np.testing.assert_allclose(orc.dense_weights(theta, 0), _printed_b(theta), rtol=0, atol=1e-15)


def test_dense_weights_end_points_and_derivatives(orc):
    np.testing.assert_array_equal(orc.dense_weights(0.0, 0), np.zeros(4))
    np.testing.assert_allclose(orc.dense_weights(1.0, 0), [1 / 6, 1 / 3, 1 / 3, 1 / 6], rtol=0, atol=1e-16)
    # U'(t^n) is the right-hand side at the first stage
    np.testing.assert_array_equal(orc.dense_weights(0.0, 1), [1.0, 0.0, 0.0, 0.0])
    h = 1e-5
    for m in (1, 2, 3):
        for th in (0.1, 0.45, 0.9):
            fd = (orc.dense_weights(th + h, m - 1) - orc.dense_weights(th - h, m - 1)) / (2 * h)
            np.testing.assert_allclose(orc.dense_weights(th, m), fd, rtol=0, atol=1e-8)


def _rk4_stages(lam, y0, h):
    """Stage right-hand sides L_j of one classical RK4 step for y' = lam y."""
    L1 = lam * y0
    L2 = lam * (y0 + 0.5 * h * L1)
    L3 = lam * (y0 + 0.5 * h * L2)
    L4 = lam * (y0 + h * L3)
    return [L1, L2, L3, L4]


def test_dense_output_order_on_linear_decay(orc):
    """One step of y' = lam y from y0 (one value per grid point, many lam): the
    dense output at theta is third order (local error ~ h^4), its derivative
    second order (~ h^3)."""
    g = grid(orc, (8, 1, 1), 0)
    lam = -np.linspace(0.5, 3.0, 8).reshape(1, 1, 1, 8)
    y0 = np.ones_like(lam)
    theta = 0.4
    errs, derrs = [], []
    for h in (0.1, 0.05, 0.025):
        L = [np.ascontiguousarray(a) for a in _rk4_stages(lam, y0, h)]
        out, dout = np.zeros_like(y0), np.zeros_like(y0)
        orc.dense_output(g, 1, theta, h, 0, y0, L, out)
        orc.dense_output(g, 1, theta, h, 1, y0, L, dout)
        exact = np.exp(lam * theta * h)
        errs.append(np.abs(out - exact).max())
        derrs.append(np.abs(dout - lam * exact).max())
    r0 = np.log2(errs[0] / errs[1]), np.log2(errs[1] / errs[2])
    r1 = np.log2(derrs[0] / derrs[1]), np.log2(derrs[1] / derrs[2])
    assert all(3.7 < r < 4.3 for r in r0), r0
    assert all(2.7 < r < 3.3 for r in r1), r1


def test_dense_output_at_theta_one_is_the_rk4_step(orc):
    g = grid(orc, (8, 1, 1), 0)
    lam = -np.linspace(0.5, 3.0, 8).reshape(1, 1, 1, 8)
    y0 = np.ones_like(lam) * 2.0
    h = 0.2
    L = [np.ascontiguousarray(a) for a in _rk4_stages(lam, y0, h)]
    out = np.zeros_like(y0)
    orc.dense_output(g, 1, 1.0, h, 0, y0, L, out)
    step = y0 + h * (L[0] + 2 * L[1] + 2 * L[2] + L[3]) / 6
    np.testing.assert_allclose(out, step, rtol=2e-16 * 8, atol=0)
