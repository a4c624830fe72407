"""Closed-form test states (test helpers; inputs only).

* gauge wave: ds^2 = -H dt^2 + H dx^2 + dy^2 + dz^2, H = 1 - A sin(2 pi (x - t)/d),
  an exact vacuum solution with harmonic slicing and zero shift;
* Schwarzschild in Kerr-Schild coordinates: stationary, so with its own lapse and
  shift d_t of gt_ij, At_ij, chi, Khat, Theta and Ghat^i vanish;
* relativistic hydrostatic slab: static fluid in alpha = exp(g x) on flat space
  with p = p0 exp(-x/L); equilibrium requires (e + p) d ln(alpha) = -dp;
* linear Alfven wave on a uniform field B0 x (v_A^2 = B0^2/(h + B0^2), App. B).
"""
import functools
import math

import numpy as np

from paper_2510_13965_amd import inputs as I

SYM = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]


def set_conformal(U, gdn, Kdn, alpha, beta, Ghat):
    """Fill the CCZ4 block of U from the physical metric, extrinsic curvature,
    lapse, shift and Ghat (arrays over the grid; gdn/Kdn shape (3,3,...))."""
    det = (gdn[0, 0] * (gdn[1, 1] * gdn[2, 2] - gdn[1, 2] * gdn[2, 1])
           - gdn[0, 1] * (gdn[1, 0] * gdn[2, 2] - gdn[1, 2] * gdn[2, 0])
           + gdn[0, 2] * (gdn[1, 0] * gdn[2, 1] - gdn[1, 1] * gdn[2, 0]))
    chi = det ** (-1.0 / 3.0)
    gup = np.linalg.inv(np.moveaxis(gdn, (0, 1), (-2, -1)))
    gup = np.moveaxis(gup, (-2, -1), (0, 1))
    K = np.einsum("ij...,ij...->...", gup, Kdn)
    for c, (i, j) in enumerate(SYM):
        U[I.GT[c]] = chi * gdn[i, j]
        U[I.AT[c]] = chi * (Kdn[i, j] - gdn[i, j] * K / 3.0)
    U[I.CHI] = chi
    U[I.KHAT] = K
    U[I.THETA] = 0.0
    for a in range(3):
        U[I.GHAT[a]] = Ghat[a]
        U[I.BETA[a]] = beta[a]
    U[I.ALPHA] = alpha


def gauge_wave(patch, A=0.1, d=1.0, t=0.0):
    Z, Y, X = patch.coords()
    ph = 2 * math.pi * (X - t) / d
    H = 1 - A * np.sin(ph)
    dtH = 2 * math.pi * A / d * np.cos(ph)
    dxH = -2 * math.pi * A / d * np.cos(ph)
    U, P, EM = I.empty_state(patch)
    z = np.zeros_like(X)
    o = np.ones_like(X)
    gdn = np.array([[H, z, z], [z, o, z], [z, z, o]])
    Kxx = -dtH / (2 * np.sqrt(H))
    Kdn = np.array([[Kxx, z, z], [z, z, z], [z, z, z]])
    Gx = 2.0 / 3.0 * H ** (-5.0 / 3.0) * dxH
    set_conformal(U, gdn, Kdn, np.sqrt(H), [z, z, z], [Gx, z, z])
    return U


@functools.lru_cache(maxsize=1)
def _kerr_schild_funcs():
    import sympy as sp

    x, y, z = sp.symbols("x y z", real=True)
    X = [x, y, z]
    M = 1
    r = sp.sqrt(x * x + y * y + z * z)
    H = M / r
    l = [x / r, y / r, z / r]
    g = sp.Matrix(3, 3, lambda i, j: (1 if i == j else 0) + 2 * H * l[i] * l[j])
    gi = sp.Matrix(3, 3, lambda i, j: (1 if i == j else 0) - 2 * H / (1 + 2 * H) * l[i] * l[j])
    alpha = 1 / sp.sqrt(1 + 2 * H)
    bu = [2 * H * l[i] / (1 + 2 * H) for i in range(3)]
    bd = [2 * H * l[i] for i in range(3)]
    dg = [[[sp.diff(g[i, j], X[k]) for j in range(3)] for i in range(3)] for k in range(3)]
    Gam = [[[sum(gi[k, m] * (dg[i][m][j] + dg[j][m][i] - dg[m][i][j]) for m in range(3)) / 2
             for j in range(3)] for i in range(3)] for k in range(3)]
    Dbeta = [[sp.diff(bd[j], X[i]) - sum(Gam[k][i][j] * bd[k] for k in range(3)) for j in range(3)]
             for i in range(3)]
    Kd = [[(Dbeta[i][j] + Dbeta[j][i]) / (2 * alpha) for j in range(3)] for i in range(3)]
    chi = (1 + 2 * H) ** sp.Rational(-1, 3)
    gt = [[chi * g[i, j] for j in range(3)] for i in range(3)]
    gtu = [[gi[i, j] / chi for j in range(3)] for i in range(3)]
    Gt = [sum(gtu[i][j] * gtu[k][l] * sp.diff(gt[j][k], X[l]) for j in range(3) for k in range(3)
              for l in range(3)) for i in range(3)]
    exprs = [g[i, j] for (i, j) in SYM] + [Kd[i][j] for (i, j) in SYM] + [alpha] + bu + Gt
    return sp.lambdify((x, y, z), exprs, modules="numpy", cse=True)


def kerr_schild(patch, killing_z=False):
    """Kerr-Schild Schwarzschild (M=1).  With killing_z the Z4 vector is the
    timelike Killing field Z^a = (d_t)^a: Theta = -n_a Z^a = alpha and
    Z_i = g_ti = beta_i, hence Z^i = beta^i; since Z is Killing and the metric is
    vacuum, R_ab + 2 nabla_(a Z_b) = 0 holds exactly (Z4 with kappa_z = 0)."""
    Z, Y, X = patch.coords()
    vals = _kerr_schild_funcs()(X, Y, Z)
    vals = [np.broadcast_to(np.asarray(v, dtype=np.float64), X.shape) for v in vals]
    gdn = np.empty((3, 3) + X.shape)
    Kdn = np.empty((3, 3) + X.shape)
    for c, (i, j) in enumerate(SYM):
        gdn[i, j] = gdn[j, i] = vals[c]
        Kdn[i, j] = Kdn[j, i] = vals[6 + c]
    U, P, EM = I.empty_state(patch)
    set_conformal(U, gdn, Kdn, vals[12], vals[13:16], vals[16:19])
    if killing_z:
        alpha = U[I.ALPHA]
        U[I.THETA] = alpha
        U[I.KHAT] = U[I.KHAT] - 2.0 * alpha
        for a in range(3):
            U[I.GHAT[a]] = U[I.GHAT[a]] + 2.0 * U[I.BETA[a]] / U[I.CHI]
    return U


def hydrostatic(patch, axis=0, g=0.1, L=1.0, p0=1e-4, B=0.0, conformal=0.0):
    """Static Gamma=2 slab along `axis`; returns U (spacetime), P, EM.
    With conformal != 0 the spatial metric is psi^4 delta_ij, psi^4 = exp(conformal*s);
    for isotropic stress the equilibrium condition does not involve psi."""
    Z, Y, X = patch.coords()
    s = (X, Y, Z)[axis]
    U, P, EM = I.empty_state(patch)
    I.flat_spacetime(U)
    U[I.ALPHA] = np.exp(g * s)
    U[I.CHI] = np.exp(-conformal * s)
    p = p0 * np.exp(-s / L)
    # e + p = p/(g L) with e = rho + p/(Gamma-1), Gamma = 2
    rho = p * (1.0 / (g * L) - 2.0)
    P[I.RHO] = rho
    P[I.EPS] = p / rho
    P[I.YE] = 0.1
    EM[axis] = B
    return U, P, EM


def alfven(patch, amp=1e-4, rho=1.0, eps=0.1, B0=0.5, t=0.0):
    """Right-moving Alfven wave along x on a Gamma=2 ideal gas at rest."""
    Z, Y, X = patch.coords()
    p = rho * eps
    h = rho * (1 + eps) + p
    vA = B0 / math.sqrt(h + B0 * B0)
    L = patch.n[0] * patch.dx[0]
    dB = amp * np.sin(2 * math.pi * (X - patch.x0[0] - vA * t) / L)
    U, P, EM = I.empty_state(patch)
    I.flat_spacetime(U)
    P[I.RHO] = rho
    P[I.EPS] = eps
    P[I.VY] = -vA / B0 * dB
    P[I.YE] = 0.1
    EM[0] = B0
    EM[1] = dB
    return U, P, EM, vA


def sound_wave(patch, amp=1e-5, rho=0.5, eps=0.1, t=0.0):
    """Right-moving linear sound wave along x (Gamma=2 ideal gas):
    c_s^2 = Gamma p / h, drho = f(x - c_s t), dv = c_s drho/rho, deps = p/rho^2 drho."""
    Z, Y, X = patch.coords()
    p = rho * eps
    h = rho * (1 + eps) + p
    cs = math.sqrt(2.0 * p / h)
    L = patch.n[0] * patch.dx[0]
    f = amp * np.sin(2 * math.pi * (X - patch.x0[0] - cs * t) / L)
    U, P, EM = I.empty_state(patch)
    I.flat_spacetime(U)
    P[I.RHO] = rho + f
    P[I.EPS] = eps + p / rho ** 2 * f
    P[I.VX] = cs * f / rho
    P[I.YE] = 0.1
    return U, P, EM, cs


def cleaning_wave(patch, amp=1e-6, c_b=1.0, t=0.0):
    """(B^x, phi) pulse moving at the cleaning speed c_b in flat space:
    B^x = f(x - c_b t), phi = c_b f(x - c_b t) (fluid at rest)."""
    Z, Y, X = patch.coords()
    L = patch.n[0] * patch.dx[0]
    f = amp * np.sin(2 * math.pi * (X - patch.x0[0] - c_b * t) / L)
    U, P, EM = I.empty_state(patch)
    I.flat_spacetime(U)
    P[I.RHO] = 1.0
    P[I.EPS] = 0.1
    P[I.YE] = 0.1
    EM[0] = f
    EM[3] = c_b * f
    return U, P, EM
