"""Pins of the oracle's IMEX(4,4,2) step with the implicit M1 collision solve
(CPU only).

* Uniform radiation relaxing in a uniform fluid at rest on flat space (F = 0,
  so J = E and the collision term is linear, dE/dt = eta - kappa_a E): one step
  multiplies the distance to equilibrium by the stability function of Table I's
  implicit tableau, R(z) = 1 + z b^T (I - z A)^-1 1 with z = -kappa_a dt, for a
  mildly stiff and a very stiff opacity.
* Without collisions the IMEX step is the explicit RK4 step of Table I.
* The implicit solves converge on rough radiation fields.
"""
import os

import numpy as np
import pytest
from fractions import Fraction

from oracle import orc
from paper_2510_13965_amd import inputs as I


def implicit_tableau():
    path = os.path.join(os.path.dirname(__file__), "golden", "table1_imex442.txt")
    lines = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    i = [k for k, l in enumerate(lines) if l[0] == "implicit_A"][0]
    A = np.array([[float(Fraction(x)) for x in lines[i + 1 + r]] for r in range(4)])
    b = np.array([float(Fraction(x)) for x in [l for l in lines if l[0] == "implicit_b"][0][1:]])
    return A, b


def uniform_state(E0, ka, eta, n=(5, 5, 5)):
    ip = I.Patch(n, (0.1,) * 3, (0.0,) * 3)
    U = np.zeros((44,) + ip.shape)
    P = np.zeros((I.NP,) + ip.shape)
    EM = np.zeros((I.NEM,) + ip.shape)
    I.flat_spacetime(U)
    P[I.RHO] = 1e-3
    P[I.EPS] = 0.1
    P[I.YE] = 0.1
    g = orc.make_grid(ip.n, ip.dx, ng=ip.ng)
    e = orc.make_eos(I.EOS_IDEAL2)
    orc.prim2con(g, e, U, P, EM, 0)
    aux = np.zeros((9,) + ip.shape)
    for s in range(3):
        U[32 + 4 * s] = E0 * (s + 1)
        aux[3 * s] = ka * (s + 1)
        aux[3 * s + 2] = eta
    return ip, g, e, U, aux


@pytest.mark.parametrize("kdt", [0.3, 10.0, 1e4])
def test_uniform_relaxation_matches_stability_function(kdt):
    E0, ka, eta, dt = 2e-5, 5e-3, 1e-7, 0.025
    ka = kdt / dt
    ip, g, e, U, aux = uniform_state(E0, ka, eta)
    par = orc.make_par(dict(I.PARAMS, evolve_m1=1, couple_matter=0))
    U1 = U.copy()
    bad = orc.imex_step(g, par, e, U1, aux, dt, periodic=True)
    assert bad == 0
    A, b = implicit_tableau()
    sl = ip.interior()
    for s in range(3):
        k = ka * (s + 1)
        z = -k * dt
        R = 1.0 + z * b @ np.linalg.solve(np.eye(4) - z * A, np.ones(4))
        yeq = eta / k
        want = yeq + R * (E0 * (s + 1) - yeq)
        got = U1[32 + 4 * s][sl]
        # the stage sums cancel by about |z|: rounding of order eps |z| E0 remains
        tol = 64 * np.finfo(float).eps * (1.0 + abs(z)) * E0 * (s + 1)
        assert np.abs(got - want).max() <= tol, (s, got.ravel()[0], want)
        assert np.abs(U1[33 + 4 * s][sl]).max() == 0.0


def test_no_collisions_is_rk4():
    ip, U, P, EM = I.perturbed_flat_state(n=8, rich=True)
    g = orc.make_grid(ip.n, ip.dx, ng=ip.ng)
    e = orc.make_eos(I.EOS_IDEAL2)
    orc.prim2con(g, e, U, P, EM, 0)
    U44, aux = I.m1_fields(ip, U, P, 77)
    aux[:] = 0.0
    par = orc.make_par(dict(I.PARAMS, evolve_m1=1))
    dt = 0.25 * ip.dx[0]
    Ui = U44.copy()
    assert orc.imex_step(g, par, e, Ui, aux, dt) == 0
    # explicit RK4 of Table I with the oracle's stage update
    Un, Us = U44.copy(), U44.copy()
    k = np.zeros_like(U44)
    acc = np.zeros_like(U44)
    Pr = np.zeros((I.NP,) + ip.shape)
    for s in range(4):
        X = Un.copy() if s == 0 else Us
        orc.con2prim(g, e, X, Pr, None, None)
        orc.rhs_full(g, par, e, X, Pr, aux, k)
        orc.rk4_stage_interior(g, 44, s, dt, Un, k, acc, Us if s < 3 else Un)
    sl = (slice(None),) + ip.interior()
    for f in range(44):
        scale = np.abs(Un[sl][f] - U44[sl][f]).max()
        d = np.abs(Ui[sl][f] - Un[sl][f]).max()
        assert d <= 1e-12 * scale + 4 * np.finfo(float).eps * np.abs(Un[sl][f]).max(), (f, d, scale)


def test_implicit_solves_converge_on_rough_fields():
    ip, U, P, EM = I.perturbed_flat_state(n=8, rich=True)
    g = orc.make_grid(ip.n, ip.dx, ng=ip.ng)
    e = orc.make_eos(I.EOS_IDEAL2)
    orc.prim2con(g, e, U, P, EM, 0)
    U44, aux = I.m1_fields(ip, U, P, 78)
    aux[0::3] *= 1e2   # stiff absorption: kappa_a up to 100
    par = orc.make_par(dict(I.PARAMS, evolve_m1=1))
    assert orc.imex_step(g, par, e, U44, aux, 0.25 * ip.dx[0]) == 0
    assert np.isfinite(U44).all()


def check_implicit_jacobian(orc):
    """App. C's printed Jacobian of the implicit M1 equation (closure frozen)
    is the derivative of its residual G: central differences approach it to
    1e-6, at second order where truncation dominates (the error drops by ~100
    from step h to h/10), on random
    states with W up to 5, flux factors 0..0.99, any Eddington factor and
    opacities up to 10."""
    r = np.random.default_rng(5)
    for t in range(200):
        A = np.eye(3) * r.uniform(1, 2) + r.uniform(-0.1, 0.1, (3, 3))
        A = 0.5 * (A + A.T)
        gd6 = np.array([A[0, 0], A[0, 1], A[0, 2], A[1, 1], A[1, 2], A[2, 2]])
        W = r.uniform(1.0, 5.0)
        d = r.normal(size=3)
        vu = d / np.sqrt(d @ A @ d) * np.sqrt(1 - 1 / W ** 2)
        E = 10 ** r.uniform(-6, -2)
        fd = r.normal(size=3)
        F = fd / np.sqrt(fd @ np.linalg.inv(A) @ fd) * E * r.uniform(0.0, 0.99)
        V = np.concatenate([[E], F])
        Vs = V * (1 + r.uniform(-0.1, 0.1, 4))
        args = (r.uniform(1 / 3, 1.0), r.uniform(0.01, 1.0), r.uniform(0.5, 1), r.uniform(0, 10), r.uniform(0, 10),
                r.uniform(0, 1e-3))
        _, Jp = orc.m1_implicit_point(gd6, vu, W, V, Vs, *args)
        err = []
        for h in (1e-5, 1e-6):
            Jf = np.zeros((4, 4))
            for c in range(4):
                dv = np.zeros(4)
                dv[c] = h * np.abs(V).sum()
                Jf[:, c] = (orc.m1_implicit_point(gd6, vu, W, V + dv, Vs, *args)[0]
                            - orc.m1_implicit_point(gd6, vu, W, V - dv, Vs, *args)[0]) / (2 * dv[c])
            err.append(np.abs(Jp - Jf).max() / np.abs(Jf).max())
        # rounding dominates below ~1e-8; above it the error is truncation
        assert min(err) <= 1e-6, (t, err)
        if err[0] > 1e-7:
            assert err[1] <= 0.05 * err[0], (t, err)


def test_implicit_jacobian_is_the_derivative():
    check_implicit_jacobian(orc)
