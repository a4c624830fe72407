"""Pins of IMEX(3,3,2) (Sec. 3.1, Table II) with the re-derived implicit half.

The printed I32L's rows sum to (0, 1, 1) against its c column (0, 1, 1/2), so
with c the row sums it is first order; the oracle's tableau keeps the printed
explicit first stage, c and b and takes the L-stable completion with equal
diagonal entries gamma = 1 - 1/sqrt(2).  Pinned here, independently of how
the tableau was derived:

* the order-2 conditions of Sec. 3.1, implicit, explicit and coupled
  (sum b = 1, sum b c = 1/2 for each pairing), with c the row sums and the
  implicit c equal to the explicit one;
* L-stability: R(z) = 1 + z b^T (I - z A)^-1 1 tends to 0 as z -> -inf,
  |R(iy)| <= 1 on the imaginary axis and R has no pole in Re z < 0; and
  R(z) - e^z = O(z^3);
* second order of the coupled scheme: the local error of a step of
  y' = lambda_E y + lambda_I y drops by 8 per halving, and the global error on
  a problem with a nonlinear explicit part and a linear implicit part with
  forcing (exact solution known, both parts nonzero along it) drops by 4, for
  mild and stiff coefficients (the printed implicit half gives 4 and 2);
* the oracle's patch step: uniform radiation at rest relaxes by the closed
  form R(z) = (1 + (1 - 2 gamma) z)/(1 - gamma z)^2 (worked by hand from the
  tableau's entries, not from the step code).
"""
import math

import numpy as np
import pytest

from oracle import orc
from paper_2510_13965_amd import inputs as I

GAMMA = 1.0 - math.sqrt(0.5)


def tab():
    return orc.imex_tableau(1)


def check_order_conditions(_=None):
    AE, AI, BE, BI = tab()
    cE, cI = AE.sum(1), AI.sum(1)
    assert np.allclose(cE, [0.0, 1.0, 0.5], atol=1e-15)
    assert np.allclose(cI, cE, atol=1e-15)
    assert np.allclose(np.triu(AE), 0.0) and np.allclose(np.triu(AI, 1), 0.0)
    for b in (BE, BI):
        assert abs(b.sum() - 1.0) <= 1e-15
        for c in (cE, cI):
            assert abs(b @ c - 0.5) <= 1e-15


def test_order_conditions():
    check_order_conditions()


def stability(z, AI, BI):
    n = len(BI)
    return 1.0 + z * BI @ np.linalg.solve(np.eye(n) - z * AI, np.ones(n))


def check_l_stability(_=None):
    AE, AI, BE, BI = tab()
    assert abs(stability(-1e9, AI, BI)) <= 1e-8
    for y in np.concatenate([np.linspace(-50, 50, 2001), np.logspace(-3, 6, 200), -np.logspace(-3, 6, 200)]):
        assert abs(stability(1j * y, AI, BI)) <= 1.0 + 1e-13, y
    d = np.diag(AI)
    assert np.all(d[d != 0] > 0)   # poles at 1/a_ii in the right half-plane
    errs = [abs(stability(z, AI, BI) - math.exp(z)) for z in (-1e-2, -5e-3)]
    assert 6.0 < errs[0] / errs[1] < 10.0   # third-order local error: ratio 8


def test_l_stability():
    check_l_stability()


def imex_R(zE, zI, AE, AI, BE, BI):
    """One IMEX step of y' = lambda_E y + lambda_I y from y = 1 (z = h lambda)."""
    n = len(BE)
    Y = np.zeros(n)
    for i in range(n):
        Y[i] = (1.0 + zE * (AE[i, :i] @ Y[:i]) + zI * (AI[i, :i] @ Y[:i])) / (1.0 - zI * AI[i, i])
    return 1.0 + (zE * BE + zI * BI) @ Y


def imex_solve(AE, AI, BE, BI, kappa, nsteps, T=1.0):
    """y' = [-y^2] + [-kappa (y - psi(t))], explicit and implicit parts in
    brackets, psi = (y' + y^2 + kappa y)/kappa of the exact solution
    y = 1 + e^-t; both parts are nonzero along the solution.  Returns the
    error at T."""
    y_ex = lambda t: 1.0 + math.exp(-t)
    psi = lambda t: (-math.exp(-t) + y_ex(t) ** 2 + kappa * y_ex(t)) / kappa
    c = AE.sum(1)
    n = len(BE)
    dt = T / nsteps
    y, t = y_ex(0.0), 0.0
    for _ in range(nsteps):
        FE, FI = np.zeros(n), np.zeros(n)
        for i in range(n):
            ti = t + c[i] * dt
            ys = y + dt * (AE[i, :i] @ FE[:i] + AI[i, :i] @ FI[:i])
            a = AI[i, i] * dt
            Y = (ys + a * kappa * psi(ti)) / (1.0 + a * kappa)
            FE[i], FI[i] = -Y * Y, -kappa * (Y - psi(ti))
        y += dt * (BE @ FE + BI @ FI)
        t += dt
    return abs(y - y_ex(T))


def check_convergence(_=None):
    AE, AI, BE, BI = tab()
    # local error of the coupled linear step: O(h^3), ratio 8 per halving
    e = [abs(imex_R(0.5 * h, -h, AE, AI, BE, BI) - math.exp(-0.5 * h)) for h in (0.02, 0.01)]
    assert 7.0 < e[0] / e[1] < 9.0, e
    for kappa in (1.0, 10.0, 1e4):
        e = [imex_solve(AE, AI, BE, BI, kappa, n) for n in (80, 160, 320)]
        rates = [math.log2(e[0] / e[1]), math.log2(e[1] / e[2])]
        assert all(1.8 < r < 2.4 for r in rates), (kappa, e, rates)


def test_second_order_convergence():
    check_convergence()


def test_printed_i32l_is_first_order():
    """The printed implicit half (rows (0,0,0), (1/2,1/2,0), (1/6,1/6,2/3)) with
    c its row sums fails sum b c = 1/2, and the coupled scheme converges at
    first order on the same problem: the reason the tableau is re-derived."""
    AE, _, BE, _ = tab()
    AIp = np.array([[0, 0, 0], [0.5, 0.5, 0], [1 / 6, 1 / 6, 2 / 3]])
    BIp = np.array([1 / 6, 1 / 6, 2 / 3])
    assert abs(BIp @ AIp.sum(1) - 5.0 / 6.0) <= 1e-15
    e = [abs(imex_R(0.5 * h, -h, AE, AIp, BE, BIp) - math.exp(-0.5 * h)) for h in (0.02, 0.01)]
    assert 3.5 < e[0] / e[1] < 4.5, e
    e = [imex_solve(AE, AIp, BE, BIp, 1.0, n) for n in (80, 160, 320)]
    assert all(0.8 < math.log2(e[k] / e[k + 1]) < 1.3 for k in range(2)), e


@pytest.mark.parametrize("kdt", [0.3, 10.0, 1e4])
def test_patch_step_relaxation_closed_form(kdt):
    check_patch_relaxation(kdt=kdt)


def check_patch_relaxation(_=None, kdt=10.0):
    """Uniform radiation at rest (flat, lapse 1, no matter coupling), energy
    absorption kappa_a and emission eta: one oracle IMEX(3,3,2) step maps E - E_eq
    to R(z) (E - E_eq), z = -kappa_a dt, R(z) = (1 + (1 - 2 gamma) z)/(1 - gamma z)^2."""
    ip = I.Patch((6, 6, 6), (0.1,) * 3, (0.0,) * 3)
    U = np.zeros((I.NU_M1,) + ip.shape)
    P = np.zeros((I.NP,) + ip.shape)
    EM = np.zeros((I.NEM,) + ip.shape)
    I.flat_spacetime(U)
    P[I.RHO], P[I.EPS], P[I.YE] = 1e-3, 0.1, 0.1
    g = orc.make_grid(ip.n, ip.dx, ng=ip.ng)
    e = orc.make_eos(I.EOS_IDEAL2)
    orc.prim2con(g, e, U, P, EM, 0)
    E0, eta, dt = 2e-5, 1e-7, 0.025
    aux = np.zeros((9,) + ip.shape)
    ka = kdt / dt
    for s in range(3):
        U[32 + 4 * s] = E0 * (s + 1)
        aux[3 * s] = ka * (s + 1)
        aux[3 * s + 2] = eta
    par = orc.make_par(dict(I.PARAMS, evolve_m1=1, couple_matter=0))
    assert orc.imex_step(g, par, e, U, aux, dt, periodic=True, scheme=1) == 0
    for s in range(3):
        k = ka * (s + 1)
        z = -k * dt
        R = (1.0 + (1.0 - 2.0 * GAMMA) * z) / (1.0 - GAMMA * z) ** 2
        want = eta / k + R * (E0 * (s + 1) - eta / k)
        got = U[32 + 4 * s][ip.interior()]
        tol = 64 * np.finfo(float).eps * (1.0 + abs(z)) * E0 * (s + 1)
        assert np.abs(got - want).max() <= tol, (kdt, s, np.abs(got - want).max(), tol)
