"""Constraint monitors on the GPU (mhd_constraints) against the oracle.

Both sides evaluate the same residuals from the same 4th-order derivatives;
the GPU collects the second derivatives of the Ricci scalar per derivative
pair and reduces the integrals in another order, so agreement is to rounding:
per field, |GPU - oracle| <= 1e-10 max|oracle| over the interior (the
residuals are differences of terms no larger than their own scale on these
states: the perturbed states have O(1/h^2) curvature noise, the star's H is
the truncation error of terms of size 16 pi E ~ 0.06, and rounding is ~1e-16
of the terms); integrals to 1e-11 relative.  The GPU's totals are the plane
rows summed in order, bit for bit, and two calls give the same bits; each
plane row is within 1e-11 of its total.
"""
import sys

import numpy as np
import pytest

from paper_2510_13965_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = 1e-10
TOL_SUM = 1e-11


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2510_13965_amd import mhd

    mhd.lib()
    return torch.device("cuda")


def prepared(orc, ip, U, P, EM):
    orc.prim2con(orc.make_grid(ip.n, ip.dx, ng=ip.ng), orc.make_eos(I.EOS_IDEAL2), U, P, EM, 0)
    return U


def gpu_constraints(ip, U):
    import torch
    from paper_2510_13965_amd import mhd

    Ud = torch.as_tensor(U).cuda()
    Cd = torch.full((5,) + ip.shape, 3.0, dtype=torch.float64, device="cuda")
    sd = torch.zeros(7 * (ip.n[2] + 1), dtype=torch.float64, device="cuda")
    mhd.constraints(mhd.patch_of(ip), Ud, Cd, sd)
    torch.cuda.synchronize()
    return Cd.cpu().numpy(), sd.cpu().numpy()


def check(orc, ip, U, tag):
    Co, so = orc.constraints(orc.make_grid(ip.n, ip.dx, ng=ip.ng), U)
    Cg, sg = gpu_constraints(ip, U)
    inter = (slice(None),) + ip.interior()
    # points outside the interior are untouched
    mask = np.ones(ip.shape, dtype=bool)
    mask[ip.interior()] = False
    assert (Cg[:, mask] == 3.0).all()
    worst = []
    for q in range(5):
        o, g = Co[inter][q], Cg[inter][q]
        m = np.abs(o).max()
        err = np.abs(g - o).max()
        worst.append(err / m if m > 0 else err)
        assert err <= TOL * m, (tag, q, err, m)
    for q in range(7):
        np.testing.assert_allclose(sg[q], so[q], rtol=TOL_SUM, atol=0, err_msg=f"{tag} sum {q}")
    # plane rows: to the same bar as their total (the pointwise bound is relative
    # to the patch's largest residual, so a plane of residuals far below it,
    # e.g. in the atmosphere, carries no relative bound of its own)
    rows = sg[7:].reshape(ip.n[2], 7)
    rows_o = so[7:].reshape(ip.n[2], 7)
    for q in range(7):
        assert np.abs(rows[:, q] - rows_o[:, q]).max() <= TOL_SUM * abs(so[q]), (tag, "plane rows", q)
    for q in range(7):
        s = 0.0
        for k in range(ip.n[2]):
            s += rows[k, q]
        assert s == sg[q], (tag, q)
    say(tag, "worst field errors relative to the field's max:", ["%.1e" % w for w in worst])
    return Cg, sg, so


def test_perturbed_rich_state(orc, dev):
    say("case constraints, perturbed flat state (rich), 32^3")
    ip, U, P, EM = I.perturbed_flat_state(rich=True)
    U = prepared(orc, ip, U, P, EM)
    Cg, sg, so = check(orc, ip, U, "rich")
    assert all(so[q] > 0 for q in range(7))  # every monitor is exercised
    # the same input gives the same bits
    Cg2, sg2 = gpu_constraints(ip, U)
    assert np.array_equal(sg, sg2) and np.array_equal(Cg, Cg2)


@pytest.mark.parametrize("n", [(37, 5, 3), (1, 1, 1), (70, 9, 4), (64, 64, 2)])
def test_ragged(orc, dev, n):
    """Partial wavefronts and blocks, a single point, thin planes."""
    say("case constraints ragged", n)
    ip = I.Patch(n, (0.2, 0.3, 0.25), (0.1, -0.2, 0.3))
    r = I.rng(78)
    U, P, EM = I.empty_state(ip)
    I.flat_spacetime(U)
    sh = ip.shape
    for c in I.GT + (I.CHI,):
        U[c] += 1e-3 * r.standard_normal(sh)
    for c in I.AT + (I.KHAT, I.THETA) + I.GHAT:
        U[c] += 1e-3 * r.standard_normal(sh)
    P[I.RHO] = 1e-3 * (1 + 0.1 * r.random(sh))
    P[I.EPS] = 0.1 * (1 + 0.1 * r.random(sh))
    for c in (I.VX, I.VY, I.VZ):
        P[c] = 0.05 * r.standard_normal(sh)
    P[I.YE] = 0.1
    EM[0:3] = 1e-3 * r.standard_normal((3,) + sh)
    EM[3] = 1e-4 * r.standard_normal(sh)
    U = prepared(orc, ip, U, P, EM)
    check(orc, ip, U, "ragged %s" % (n,))


def test_two_ghosts_and_padded_strides(orc, dev):
    """The minimum ghost width (the stencils reach exactly two points out) and a
    layout with padded row, plane and field strides; the padding is untouched."""
    import torch
    from paper_2510_13965_amd import mhd

    say("case constraints, ng = 2, padded strides")
    ip = I.Patch((21, 6, 5), (0.2, 0.3, 0.25), (0.0, 0.0, 0.0), 2)
    r = I.rng(79)
    U, P, EM = I.empty_state(ip)
    I.flat_spacetime(U)
    sh = ip.shape
    for c in I.GT + (I.CHI,) + I.AT + (I.KHAT, I.THETA) + I.GHAT:
        U[c] += 1e-3 * r.standard_normal(sh)
    P[I.RHO] = 1e-3 * (1 + 0.1 * r.random(sh))
    P[I.EPS] = 0.1 * (1 + 0.1 * r.random(sh))
    for c in (I.VX, I.VY, I.VZ):
        P[c] = 0.05 * r.standard_normal(sh)
    P[I.YE] = 0.1
    EM[0:3] = 1e-3 * r.standard_normal((3,) + sh)
    EM[3] = 1e-4 * r.standard_normal(sh)
    U = prepared(orc, ip, U, P, EM)
    Co, so = orc.constraints(orc.make_grid(ip.n, ip.dx, ng=ip.ng), U)
    Nz, Ny, Nx = sh
    sy, sz = Nx + 3, (Nx + 3) * (Ny + 1)
    sf = sz * Nz + 11

    def padded(a):
        buf = np.full(a.shape[0] * sf, np.nan)
        v = np.lib.stride_tricks.as_strided(buf, shape=a.shape, strides=(sf * 8, sz * 8, sy * 8, 8))
        v[...] = a
        return buf, v

    Ub, _ = padded(U)
    Cb, _ = padded(np.full((5,) + sh, 3.0))
    Ud, Cd = torch.as_tensor(Ub).cuda(), torch.as_tensor(Cb).cuda()
    sd = torch.zeros(7 * (ip.n[2] + 1), dtype=torch.float64, device="cuda")
    mhd.constraints(mhd.patch_of(ip, strides=(sy, sz, sf)), Ud, Cd, sd)
    torch.cuda.synchronize()
    cb = Cd.cpu().numpy()
    Cg = np.lib.stride_tricks.as_strided(cb, shape=(5,) + sh, strides=(sf * 8, sz * 8, sy * 8, 8)).copy()
    inter = (slice(None),) + ip.interior()
    for q in range(5):
        m = np.abs(Co[inter][q]).max()
        assert np.abs(Cg[inter][q] - Co[inter][q]).max() <= TOL * m, q
    mask = np.ones(sh, dtype=bool)
    mask[ip.interior()] = False
    assert (Cg[:, mask] == 3.0).all()
    # the padding between rows, planes and fields is never written
    written = np.zeros(cb.shape, dtype=bool)
    np.lib.stride_tricks.as_strided(written, shape=(5,) + sh, strides=(sf, sz, sy, 1))[...] = True
    assert np.isnan(cb[~written]).all()
    np.testing.assert_allclose(sd.cpu().numpy(), so, rtol=TOL_SUM, atol=TOL_SUM * np.abs(so).max())


@pytest.mark.parametrize("n", [32, 128])
def test_tov_star(orc, dev, n):
    """The TOV star (isotropic coordinates, K_ij = 0): H is the truncation error
    of the initial data; the baryonic mass of the K = 100, Gamma = 2,
    rho_c = 1.28e-3 star is 1.506 to three digits once resolved."""
    say("case constraints TOV star", n)
    ip, U, P, EM = I.tov_star_state(n=n)
    U = prepared(orc, ip, U, P, EM)
    Cg, sg, so = check(orc, ip, U, "star %d" % n)
    if n == 128:
        assert abs(sg[2] - 1.506) < 2e-3, sg[2]


def test_baryonic_mass_conserved_on_a_periodic_patch(orc, dev):
    """The fluid update is in flux form: on a periodic patch the fluxes of the
    conserved density telescope and the baryonic mass is constant up to
    rounding (the oracle's own RK4 step keeps it to 2e-16 on this state).
    Three GPU steps, the monitor read through the driver."""
    import torch
    from paper_2510_13965_amd.step import PatchRun

    say("case constraints: baryonic mass over three periodic RK4 steps")
    ip, U, P, EM = I.perturbed_flat_state(rich=True)
    U = prepared(orc, ip, U, P, EM)
    run = PatchRun(ip, U, I.EOS_IDEAL2, I.PARAMS, periodic=True)
    masses = []
    for it in range(4):
        if it == 0:
            # the driver's monitor call gives the same integrals as the direct one
            torch.cuda.synchronize()
            _, s = gpu_constraints(ip, run.Un.cpu().numpy())
            mon = run.monitors()
            assert [mon[k] for k in ("H2", "M2", "baryon_mass", "Theta2", "Z2", "phi2", "B2")] == list(s[:7])
        masses.append(run.monitors()["baryon_mass"])
        run.step(0.25 * ip.dx[0])
    torch.cuda.synchronize()
    assert bool(torch.isfinite(run.Un).all().item())
    m0 = masses[0]
    assert all(abs(m - m0) <= 1e-14 * m0 for m in masses), masses
    say("baryonic mass over the steps", masses)


def test_level_monitors_per_box(orc, dev):
    """LevelRun.monitors: one entry per box, equal to the direct call on that box."""
    from paper_2510_13965_amd.step import MONITORS, LevelRun

    say("case constraints: level monitors per box")
    ip1, U1, P1, EM1 = I.perturbed_flat_state(rich=True, n=16)
    U1 = prepared(orc, ip1, U1, P1, EM1)
    ip2, U2, P2, EM2 = I.tov_star_state(n=32)
    U2 = prepared(orc, ip2, U2, P2, EM2)
    run = LevelRun([ip1, ip2], [U1, U2], I.EOS_IDEAL2, I.PARAMS)
    mons = run.monitors()
    assert len(mons) == 2
    for ip, U, m in ((ip1, U1, mons[0]), (ip2, U2, mons[1])):
        _, s = gpu_constraints(ip, U)
        assert [m[k] for k in MONITORS] == list(s[:7])


def test_rejects_bad_arguments(dev):
    import torch
    from paper_2510_13965_amd import mhd

    say("case constraints argument checks")
    ip = I.Patch((8, 8, 8), (0.25,) * 3, (0.0,) * 3, 1)
    U = torch.zeros((32,) + ip.shape, dtype=torch.float64, device="cuda")
    Cd = torch.zeros((5,) + ip.shape, dtype=torch.float64, device="cuda")
    s = torch.zeros(7 * 9, dtype=torch.float64, device="cuda")
    with pytest.raises(mhd.MhdError, match="ghost width must be >= 2"):
        mhd.constraints(mhd.patch_of(ip), U, Cd, s)
    ip = I.Patch((8, 8, 8), (0.25,) * 3, (0.0,) * 3, 3)
    U = torch.zeros((32,) + ip.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(mhd.MhdError, match="must not alias"):
        mhd.constraints(mhd.patch_of(ip), U, U, s)
