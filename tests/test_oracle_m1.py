"""Pins of the oracle's grey M1 part (CPU only).

Closure: the Eddington factor's end points; v = 0 gives xi = |F|/E; radiation
isotropic in the fluid frame (the thick limit, exact for the Minerbo closure)
gives xi = 0 and the boosted isotropic stress; a single beam (the thin limit,
also exact) gives xi = 1 and P_ij = E l_i l_j, for moving fluids too.
Interface fluxes: a linear profile is differentiated exactly (limiter at 1), a
constant one gives zero, an odd-even pattern falls back to the Lax-Friedrichs
flux with A = 1, a large opacity switches the diffusion off.
Sources: v = 0 collision terms in closed form; the fluid loses exactly what
the radiation gains; the CCZ4 matter terms gain the radiation's E, F_i, P_ij.
"""
import math

import numpy as np
import pytest

from oracle import orc
from paper_2510_13965_amd import inputs as I

FLAT = np.array([1.0, 0, 0, 1.0, 0, 1.0])


def test_eddington_end_points():
    assert orc.m1_eddington(0.0) == pytest.approx(1.0 / 3.0, abs=1e-16)
    assert orc.m1_eddington(1.0) == pytest.approx(1.0, abs=1e-15)
    xs = np.linspace(0, 1, 101)
    ch = [orc.m1_eddington(x) for x in xs]
    assert np.all(np.diff(ch) > 0)


@pytest.mark.parametrize("ratio", [0.0, 0.1, 0.5, 0.9, 0.999])
def test_closure_at_rest_xi_is_flux_ratio(ratio):
    E = 2e-5
    F = np.array([0.6, -0.8, 0.0]) * ratio * E
    xi, chi, P, J, H, it = orc.m1_closure(E, F, np.zeros(3), 1.0, FLAT, FLAT)
    assert xi == pytest.approx(ratio, rel=1e-13, abs=1e-15)
    assert J == pytest.approx(E, rel=1e-14)
    assert np.allclose(H, F, rtol=1e-14, atol=1e-30)
    dthick = 1.5 * (1 - chi)
    F2 = F @ F
    thin = np.outer(F, F) / F2 * E if F2 > 0 else np.zeros((3, 3))
    want = (1 - dthick) * thin + dthick * E / 3 * np.eye(3)
    got = P[[0, 1, 2, 1, 3, 4, 2, 4, 5]].reshape(3, 3)
    assert np.allclose(got, want, rtol=1e-13, atol=1e-25)


def metric(seed):
    r = np.random.default_rng(seed)
    A = np.eye(3) + 0.15 * r.normal(size=(3, 3))
    g = A @ A.T
    return g, np.linalg.inv(g)


def pack(M):
    return np.array([M[0, 0], M[0, 1], M[0, 2], M[1, 1], M[1, 2], M[2, 2]])


def test_closure_comoving_isotropic_is_thick():
    g, gi = metric(3)
    v = np.array([0.3, -0.2, 0.25])
    W = 1 / math.sqrt(1 - v @ g @ v)
    vd = g @ v
    J0 = 3e-6
    E = J0 * (4 * W * W - 1) / 3
    F = 4.0 / 3.0 * J0 * W * W * vd
    xi, chi, P, J, H, it = orc.m1_closure(E, F, v, W, pack(g), pack(gi))
    assert xi == pytest.approx(0.0, abs=1e-7)
    assert J == pytest.approx(J0, rel=1e-12)
    want = 4.0 / 3.0 * J0 * W * W * np.outer(vd, vd) + J0 / 3 * g
    assert np.allclose(P, pack(want), rtol=1e-10, atol=1e-12 * J0)


@pytest.mark.parametrize("vmag", [0.0, 0.4, 0.8])
def test_closure_beam_is_thin(vmag):
    g, gi = metric(4)
    l = np.array([0.2, 1.0, -0.4])          # beam direction, lower index, unit length
    l = l / math.sqrt(l @ gi @ l)
    E = 1e-5
    F = E * l
    vdir = np.array([1.0, 0.5, 0.2])
    v = vdir / math.sqrt(vdir @ g @ vdir) * vmag
    W = 1 / math.sqrt(1 - v @ g @ v)
    xi, chi, P, J, H, it = orc.m1_closure(E, F, v, W, pack(g), pack(gi))
    assert xi == pytest.approx(1.0, abs=1e-9)
    assert np.allclose(P, pack(E * np.outer(l, l)), rtol=1e-9, atol=1e-14 * E)


# ---------------------------------------------------------------- patch-level checks

def flat_patch(n=(8, 6, 6), dx=0.1):
    ip = I.Patch(n, (dx,) * 3, (0.0,) * 3)
    U = np.zeros((44,) + ip.shape)
    P = np.zeros((I.NP,) + ip.shape)
    I.flat_spacetime(U)
    P[I.RHO] = 1e-3
    P[I.EPS] = 0.1
    P[I.PRESS] = 1e-4
    P[I.WLOR] = 1.0
    U[I.DBAR] = 1e-3
    U[I.TAUBAR] = 1e-4
    aux = np.zeros((9,) + ip.shape)
    return ip, U, P, aux


def m1_only(ip, U, P, aux):
    g = orc.make_grid(ip.n, ip.dx, ng=ip.ng)
    par = dict(I.PARAMS, evolve_m1=1)
    out = np.zeros_like(U)
    orc.rhs_full(g, orc.make_par(par), orc.make_eos(I.EOS_IDEAL2), U, P, aux, out)
    return out[(slice(None),) + ip.interior()]


def test_uniform_radiation_collisions_closed_form():
    ip, U, P, aux = flat_patch()
    E, Fx = 2e-5, 0.5e-5
    for s in range(3):
        U[32 + 4 * s] = E * (1 + s)
        U[33 + 4 * s] = Fx * (1 + s)
        aux[3 * s] = 1e-3 * (s + 1)      # kappa_a
        aux[3 * s + 1] = 2e-3            # kappa_s
        aux[3 * s + 2] = 3e-8            # eta
    r = m1_only(ip, U, P, aux)
    tot_E, tot_F = 0.0, 0.0
    for s in range(3):
        ka, ks, eta = 1e-3 * (s + 1), 2e-3, 3e-8
        Es, Fs = E * (1 + s), Fx * (1 + s)
        assert np.allclose(r[32 + 4 * s], eta - ka * Es, rtol=1e-12, atol=0)
        assert np.allclose(r[33 + 4 * s], -(ka + ks) * Fs, rtol=1e-12, atol=0)
        assert np.abs(r[34 + 4 * s]).max() == 0.0
        tot_E += eta - ka * Es
        tot_F += -(ka + ks) * Fs
    # what the radiation gains the fluid loses (the fluid part is zero here)
    assert np.allclose(r[I.TAUBAR], -tot_E, rtol=1e-12)
    assert np.allclose(r[I.SBAR[0]], -tot_F, rtol=1e-12)


def beam_along_x(E_of_x, ip, U):
    Z, Y, X = ip.coords()
    E = E_of_x(X)
    U[32] = E
    U[33] = E          # |F| = E along x: a beam, thin closure


def test_linear_beam_profile_differentiated_exactly():
    ip, U, P, aux = flat_patch()
    beam_along_x(lambda x: 1e-5 * (1.0 + 0.3 * x), ip, U)
    r = m1_only(ip, U, P, aux)
    # E_t = -d_x F^x = -0.3e-5, F_t = -d_x P^x_x = -0.3e-5 (P_xx = E for the beam)
    assert np.allclose(r[32], -0.3e-5, rtol=1e-9)
    assert np.allclose(r[33], -0.3e-5, rtol=1e-9)
    assert np.abs(r[34]).max() <= 1e-20 and np.abs(r[35]).max() <= 1e-20


def test_constant_beam_has_zero_flux_difference():
    ip, U, P, aux = flat_patch()
    beam_along_x(lambda x: 1e-5 + 0 * x, ip, U)
    r = m1_only(ip, U, P, aux)
    assert np.abs(r[32]).max() == 0.0 and np.abs(r[33]).max() == 0.0


def test_odd_even_pattern_gets_lax_friedrichs():
    """u_i = a (1 + b (-1)^i): limiter 0, A forced to 1, so F^ = F^LO and the
    RHS is the LF difference: -(F_i+1 - F_i-1)/(2dx) + lambda (u_i+1 - 2u_i + u_i-1)/(2dx)."""
    ip, U, P, aux = flat_patch()
    Z, Y, X = ip.coords()
    i = np.rint(X / ip.dx[0]).astype(int)
    a, b = 1e-5, 0.2
    U[32] = a * (1 + b * (-1.0) ** i)
    U[33] = U[32]
    aux[0] = 50.0        # large opacity: A = tanh(1/(kappa dx)) ~ 0.2 unless forced to 1
    r = m1_only(ip, U, P, aux)
    E = U[32][ip.interior()]
    # beam: flux of E is E, lambda = 1 (thin speed |F^x|/|F| = 1, E|F^x|/F^2 = 1)
    Ep = np.roll(U[32], -1, axis=2)[ip.interior()]
    Em = np.roll(U[32], 1, axis=2)[ip.interior()]
    want = -(Ep - Em) / (2 * ip.dx[0]) + (Ep - 2 * E + Em) / (2 * ip.dx[0])
    got = r[32] - (-aux[0][ip.interior()] * E)   # remove the absorption term eta - kappa_a J (eta = 0, J = E)
    assert np.allclose(got, want, rtol=1e-9, atol=1e-9 * a / ip.dx[0])


def test_high_opacity_turns_off_diffusion():
    """A jump with kappa dx >> 1: A = tanh(1/(kappa dx)) ~ 1e-3, so the RHS is the
    centred HO difference up to A times the Lax-Friedrichs diffusion."""
    ip, U, P, aux = flat_patch()
    Z, Y, X = ip.coords()
    E = np.where(X < 0.35, 1e-5, 2e-5)
    U[32] = E
    U[33] = 0.5 * E
    kap = 1e4
    aux[1] = kap           # scattering only: no absorption source on E
    r = m1_only(ip, U, P, aux)
    A = math.tanh(1.0 / (kap * ip.dx[0]))
    f = 0.5 * E            # flux of Ebar along x: alpha Fbar^x
    fp = np.roll(f, -1, axis=2)[ip.interior()]
    fm = np.roll(f, 1, axis=2)[ip.interior()]
    r_ho = -(fp - fm) / (2 * ip.dx[0])
    lam_max = 1.0
    bound = A * lam_max * 1e-5 / ip.dx[0]
    d = np.abs(r[32] - r_ho)
    assert d.max() <= 1.01 * bound
    assert d.max() > 0.1 * bound        # the diffusive part is small, not absent
    assert np.abs(r[32][:, :, 0]).max() == 0.0 and np.abs(r[32][:, :, -1]).max() == 0.0


def test_matter_terms_gain_radiation():
    """Flat space, fluid at rest: the CCZ4 matter terms change by the radiation's
    E, F_i, P_ij: dK = 4 pi (E + tr P), dTheta = -8 pi E, dGhat^i = -16 pi F_i,
    dAt_ij = -8 pi P_ij^TF (alpha = chi = 1)."""
    ip, U, P, aux = flat_patch()
    g = orc.make_grid(ip.n, ip.dx, ng=ip.ng)
    e = orc.make_eos(I.EOS_IDEAL2)
    par0 = orc.make_par(dict(I.PARAMS, evolve_m1=1))
    base = np.zeros_like(U)
    orc.rhs_full(g, par0, e, U, P, aux, base)
    E, F = 3e-6, np.array([1e-6, -0.5e-6, 0.2e-6])
    U[32] = E
    U[33:36] = F[:, None, None, None]
    out = np.zeros_like(U)
    orc.rhs_full(g, par0, e, U, P, aux, out)
    d = (out - base)[(slice(None),) + ip.interior()]
    xi, chi, Pij, J, H, it = orc.m1_closure(E, F, np.zeros(3), 1.0, FLAT, FLAT)
    Pm = Pij[[0, 1, 2, 1, 3, 4, 2, 4, 5]].reshape(3, 3)
    trP = np.trace(Pm)
    pi = math.pi
    assert np.allclose(d[I.KHAT], 4 * pi * (E + trP), rtol=1e-10)
    assert np.allclose(d[I.THETA], -8 * pi * E, rtol=1e-10)
    for a in range(3):
        assert np.allclose(d[I.GHAT[a]], -16 * pi * F[a], rtol=1e-10)
    TF = Pm - trP / 3 * np.eye(3)
    for c, (a, b) in enumerate([(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]):
        assert np.allclose(d[I.AT[c]], -8 * pi * TF[a, b], rtol=1e-9, atol=1e-20)


def thick_uniform(ip, U, Ebar=2e-5):
    U[32] = Ebar       # F = 0, v = 0: thick closure, P^i_j = E/3 delta
    return Ebar


def test_lapse_gradient_source():
    """alpha = 1 + a x: F_x gains -d_x(alpha Ebar/3) - Ebar d_x alpha = -(4/3) a Ebar."""
    ip, U, P, aux = flat_patch()
    Z, Y, X = ip.coords()
    a = 0.05
    U[I.ALPHA] = 1.0 + a * X
    Eb = thick_uniform(ip, U)
    r = m1_only(ip, U, P, aux)
    assert np.allclose(r[33], -4.0 / 3.0 * a * Eb, rtol=1e-11)
    assert np.abs(r[32]).max() <= 1e-25


def test_shift_gradient_source():
    """beta^x = b y, uniform Fbar: F_y gains Fbar_x d_y beta^x = b Fbar_x."""
    ip, U, P, aux = flat_patch()
    Z, Y, X = ip.coords()
    b = 0.03
    U[I.BETA[0]] = b * Y
    U[32] = 2e-5
    U[33] = 0.5e-5
    r = m1_only(ip, U, P, aux)
    assert np.allclose(r[34], b * 0.5e-5, rtol=1e-11)


def test_extrinsic_curvature_source():
    """Uniform At_xx and Khat: Ebar gains (alpha/chi) Pbar^ij At_ij + alpha/3 tr Pbar Khat."""
    ip, U, P, aux = flat_patch()
    U[I.AT[0]] = 0.01
    U[I.KHAT] = 0.02
    E, F = 3e-5, np.array([1e-5, 0.4e-5, 0.0])
    U[32] = E
    U[33:36] = F[:, None, None, None]
    r = m1_only(ip, U, P, aux)
    xi, chi, Pij, J, H, it = orc.m1_closure(E, F, np.zeros(3), 1.0, FLAT, FLAT)
    want = Pij[0] * 0.01 + (Pij[0] + Pij[3] + Pij[5]) / 3.0 * 0.02
    assert np.allclose(r[32], want, rtol=1e-11)


def test_conformal_factor_and_metric_gradient_sources():
    """chi = 1 + c x: F_x gains -(alpha/2chi) tr Pbar d_x chi = -Ebar c/(2 chi);
    gt_xx = 1 + d x: F_x gains (alpha/2chi) Pbar^xx d_x gt_xx = Ebar d / (6 gt_xx)."""
    ip, U, P, aux = flat_patch()
    Z, Y, X = ip.coords()
    c = 0.04
    U[I.CHI] = 1.0 + c * X
    Eb = thick_uniform(ip, U)
    r = m1_only(ip, U, P, aux)
    chi = (1.0 + c * X)[ip.interior()]
    assert np.allclose(r[33], -Eb * c / (2 * chi), rtol=1e-11)
    ip, U, P, aux = flat_patch()
    Z, Y, X = ip.coords()
    d = 0.05
    U[I.GT[0]] = 1.0 + d * X
    Eb = thick_uniform(ip, U)
    r = m1_only(ip, U, P, aux)
    gxx = (1.0 + d * X)[ip.interior()]
    assert np.allclose(r[33], Eb * d / (6 * gxx), rtol=1e-11)
