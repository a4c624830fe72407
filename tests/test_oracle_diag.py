"""Pins of the oracle's constraint monitors (energy and momentum constraints,
Z4 variables, volume integrals) against closed forms.

* Conformally flat metric gamma = psi^4 delta, K_ij = 0, no matter: the energy
  constraint is the Ricci scalar, R = -8 psi^-5 Laplacian(psi); 4th-order
  convergence to it.
* The slice t = f(x, y, z) of flat spacetime: gamma_ij = delta_ij - f_i f_j,
  K_ij = -f_ij / sqrt(1 - |grad f|^2).  A vacuum solution, so H = M_i = 0; the
  residuals converge to zero at 4th order.  The metric is not conformally flat
  and K_ij is not pure trace, so every term of both constraints is exercised.
* Flat conformal metric, constant chi, K = 0: H = -16 pi E and M_i = -8 pi S_i
  exactly, with E, S_i the densitized fields over sqrt(gamma) = chi^-3/2.
* gt = diag(e^u, e^-u, 1), u = u(x): Gt^x = u' e^-u, so with Ghat = 0,
  Z_i Z^i = chi u'^2 e^-u / 4 up to the 4th-order error of Gt.
* Integrals of a Gaussian density, of phi^2 and of B^2 against their closed
  forms; the totals are the sums of the per-plane rows.
"""
import math

import numpy as np
import pytest

NU = 32
PI = math.pi


@pytest.fixture(scope="module")
def orc():
    from oracle import orc as O

    O.lib()
    return O


def coords(n, h, ng=3, x0=0.0):
    """padded coordinates (z, y, x) broadcastable arrays of a cube of n interior
    points per axis starting at x0"""
    x = x0 + (np.arange(n + 2 * ng) - ng) * h
    return x[None, None, :], x[None, :, None], x[:, None, None]


def base(n):
    U = np.zeros((NU,) + (n + 6,) * 3)
    for f in (0, 3, 5):
        U[f] = 1.0
    U[12] = 1.0
    U[18] = 1.0
    return U


def interior(a, ng=3):
    return a[..., ng:-ng, ng:-ng, ng:-ng]


def conformally_flat(orc, n, L=4.0):
    h = L / n
    X, Y, Z = coords(n, h, x0=-L / 2 + h / 2)
    r2 = X * X + Y * Y + Z * Z
    A, s = 0.2, 1.0
    e = np.exp(-r2 / s ** 2)
    psi = 1.0 + A * e
    lap = A * e * (4.0 * r2 / s ** 4 - 6.0 / s ** 2)
    U = base(n)
    U[12] = psi ** -4
    C, _ = orc.constraints(orc.make_grid((n,) * 3, (h,) * 3), U)
    exact = -8.0 * psi ** -5 * lap
    return np.abs(interior(C[0] - exact)).max(), np.abs(interior(C[1:4])).max(), np.abs(interior(exact)).max()


def test_conformally_flat_ricci_scalar(orc):
    e1, m1, scale = conformally_flat(orc, 16)
    e2, m2, _ = conformally_flat(orc, 32)
    assert e2 < 0.05 * scale
    assert 10.0 < e1 / e2 < 24.0, (e1, e2)  # 4th order: 16
    assert m1 == 0.0 and m2 == 0.0  # K_ij = 0, no momentum


def minkowski_slice(orc, n, L=4.0):
    h = L / n
    X, Y, Z = coords(n, h, x0=-L / 2 + h / 2)
    a, s = 0.3, 1.0
    e = np.exp(-(X * X + Y * Y + Z * Z) / s ** 2)
    xs = (X, Y, Z)
    shape = (n + 6,) * 3
    f1 = [np.broadcast_to(-2.0 * xs[i] / s ** 2 * a * e, shape) for i in range(3)]
    f2 = [[np.broadcast_to(a * e * (4.0 * xs[i] * xs[j] / s ** 4 - (2.0 / s ** 2 if i == j else 0.0)), shape)
           for j in range(3)] for i in range(3)]
    g2 = f1[0] ** 2 + f1[1] ** 2 + f1[2] ** 2
    assert g2.max() < 0.2
    lapse = np.sqrt(1.0 - g2)
    gdn = [[(1.0 if i == j else 0.0) - f1[i] * f1[j] for j in range(3)] for i in range(3)]
    gup = [[(1.0 if i == j else 0.0) + f1[i] * f1[j] / (1.0 - g2) for j in range(3)] for i in range(3)]
    Kdn = [[-f2[i][j] / lapse for j in range(3)] for i in range(3)]
    K = sum(gup[i][j] * Kdn[i][j] for i in range(3) for j in range(3))
    chi = (1.0 - g2) ** (-1.0 / 3.0)  # det gamma = 1 - |grad f|^2
    U = base(n)
    S6 = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    for q, (i, j) in enumerate(S6):
        U[q] = chi * gdn[i][j]
        U[6 + q] = chi * (Kdn[i][j] - gdn[i][j] * K / 3.0)
    U[12] = chi
    U[13] = K
    C, _ = orc.constraints(orc.make_grid((n,) * 3, (h,) * 3), U)
    # scale of the individual terms of H: K_ij K^ij
    KK = sum(Kdn[i][j] * Kdn[k][l] * gup[i][k] * gup[j][l] for i in range(3) for j in range(3) for k in range(3)
             for l in range(3))
    return np.abs(interior(C[0])).max(), np.abs(interior(C[1:4])).max(), np.abs(KK).max()


def test_minkowski_slice_is_a_vacuum_solution(orc):
    # h = 1/8 and 1/16 of the Gaussian's width (at 1/4 the momentum residual
    # is still pre-asymptotic: ratio 9 instead of 16)
    H1, M1, scale = minkowski_slice(orc, 32)
    H2, M2, _ = minkowski_slice(orc, 64)
    assert H2 < 0.01 * scale and M2 < 0.01 * scale, (H2, M2, scale)
    assert 10.0 < H1 / H2 < 24.0, (H1, H2)
    assert 10.0 < M1 / M2 < 24.0, (M1, M2)


def test_matter_terms_exact(orc):
    n, h = 8, 0.5
    r = np.random.default_rng(3)
    U = base(n)
    chi = 0.8
    for f in (0, 3, 5):
        U[f] = 1.0
    U[12] = chi
    U[22] = r.uniform(0.1, 1.0, U[22].shape)
    U[24] = r.uniform(0.0, 0.5, U[24].shape)
    for i in range(3):
        U[25 + i] = r.normal(size=U[22].shape)
    C, _ = orc.constraints(orc.make_grid((n,) * 3, (h,) * 3), U)
    sg = chi ** -1.5
    E = (U[24] + U[22]) / sg
    np.testing.assert_allclose(interior(C[0]), interior(-16.0 * PI * E), rtol=1e-13, atol=0)
    for i in range(3):
        np.testing.assert_allclose(interior(C[1 + i]), interior(-8.0 * PI * U[25 + i] / sg), rtol=1e-13, atol=0)


def z_case(orc, n, L=4.0):
    h = L / n
    X, _, _ = coords(n, h)
    shape = (n + 6,) * 3
    u = np.broadcast_to(0.2 * np.sin(X), shape)
    du = np.broadcast_to(0.2 * np.cos(X), shape)
    U = base(n)
    chi = 0.7
    U[0] = np.exp(u)
    U[3] = np.exp(-u)
    U[12] = chi
    C, _ = orc.constraints(orc.make_grid((n,) * 3, (h,) * 3), U)
    exact = chi * du ** 2 * np.exp(-u) / 4.0
    return np.abs(interior(C[4] - exact)).max(), np.abs(exact).max()


def test_z_from_the_metric(orc):
    e1, scale = z_case(orc, 16)
    e2, _ = z_case(orc, 32)
    assert e2 < 1e-4 * scale
    assert 10.0 < e1 / e2 < 24.0, (e1, e2)


def test_integrals_and_plane_rows(orc):
    n, L = 40, 10.0
    h = L / n
    X, Y, Z = coords(n, h, x0=-L / 2 + h / 2)
    r2 = X * X + Y * Y + Z * Z
    s = 1.0
    U = base(n)
    chi = 0.8
    U[12] = chi
    sg = chi ** -1.5
    U[22] = 1e-3 * np.exp(-r2 / s ** 2)
    U[14] = 0.01 * np.exp(-r2 / (2 * s ** 2))  # Theta^2 integrates like the density
    U[31] = sg * 0.5 * np.exp(-r2 / (2 * s ** 2))
    U[28] = sg * 0.3
    U[15] = 0.2  # Ghat^x: Z^x = chi Ghat^x / 2 on the flat conformal metric
    g = orc.make_grid((n,) * 3, (h,) * 3)
    C, sums = orc.constraints(g, U)
    gauss = (PI ** 0.5 * s) ** 3  # integral of exp(-r^2/s^2)
    np.testing.assert_allclose(sums[2], 1e-3 * gauss, rtol=1e-9)
    np.testing.assert_allclose(sums[3], 1e-4 * gauss, rtol=1e-9)
    np.testing.assert_allclose(sums[5], 0.25 * gauss, rtol=1e-9)
    np.testing.assert_allclose(sums[6], 0.09 / chi * L ** 3, rtol=1e-12)
    np.testing.assert_allclose(sums[4], chi * 0.04 / 4.0 * L ** 3, rtol=1e-12)
    rows = sums[7:].reshape(n, 7)
    np.testing.assert_allclose(rows.sum(axis=0), sums[:7], rtol=1e-13)
    # H^2 and M^2 rows are the volume sums of the residual fields
    dV = h ** 3
    np.testing.assert_allclose(sums[0], (interior(C[0]) ** 2).sum() * dV, rtol=1e-12)
    np.testing.assert_allclose(sums[1], (interior(C[1:4]) ** 2).sum() * dV, rtol=1e-12)
    np.testing.assert_allclose(rows[:, 2], (interior(U[22])).sum(axis=(1, 2)) * dV, rtol=1e-12)
