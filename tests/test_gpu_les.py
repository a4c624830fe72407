"""GPU parity of the gradient SGS (LES) term of the induction equation
(App. A, C_M = 8) against the FP64 oracle: the whole right-hand side (per
field, max |G - O| / max |O| <= 1e-10) and the term itself, isolated as the
difference of the right-hand sides with and without it (1e-10 of its own
largest value), on the perturbed flat patch (periodic, every field
perturbed) and on the star with a seeded flow.
"""
import sys

import numpy as np
import pytest

from paper_2510_13965_amd import inputs as I

pytestmark = pytest.mark.gpu


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


def both(orc, ip, U, par_cfg):
    import torch
    from paper_2510_13965_amd.step import PatchRun

    g = orc.make_grid(ip.n, ip.dx, ng=ip.ng)
    e = orc.make_eos(I.EOS_IDEAL2)
    Uo = U.copy()
    Po = np.zeros((I.NP,) + ip.shape)
    orc.con2prim(g, e, Uo, Po, None, None)
    O = np.zeros_like(U)
    orc.rhs(g, orc.make_par(par_cfg), e, Uo, Po, O)
    r = PatchRun(ip, U, I.EOS_IDEAL2, par_cfg)
    r.rhs_eval(r.Un)
    torch.cuda.synchronize()
    return r.k.cpu().numpy(), O


def flow(ip, P):
    """The static star has v = 0, where the SGS term vanishes: give its matter
    a smooth rotation about z plus a shear, tapered by rho/rho_max (up to 0.05)."""
    Z, Y, X = ip.coords()
    w = P[I.RHO] / P[I.RHO].max()
    P[3] += 0.02 * w * (-Y + 0.3 * np.sin(0.4 * Z))
    P[4] += 0.02 * w * (X + 0.2 * np.cos(0.3 * Z))
    P[5] += 0.01 * w * np.sin(0.3 * X) * np.cos(0.2 * Y)


@pytest.mark.parametrize("case", ["flat", "star"])
def test_les_rhs_parity(orc, dev, case):
    if case == "flat":
        say("case les rhs, perturbed flat 20^3")
        ip, U, P, EM = I.perturbed_flat_state(n=20, rich=True)
    else:
        say("case les rhs, star 40^3 with a seeded flow")
        ip, U, P, EM = I.tov_star_state(n=40)
        flow(ip, P)
    g = orc.make_grid(ip.n, ip.dx, ng=ip.ng)
    orc.prim2con(g, orc.make_eos(I.EOS_IDEAL2), U, P, EM, 0)
    G8, O8 = both(orc, ip, U, dict(I.PARAMS, les_cm=8.0))
    G0, O0 = both(orc, ip, U, I.PARAMS)
    sl = (slice(None),) + ip.interior()
    for f in range(I.NU):
        m = np.abs(O8[sl][f]).max()
        if m > 0:
            assert np.abs(G8[sl][f] - O8[sl][f]).max() <= 1e-10 * m, (case, f)
    for f in (28, 29, 30):
        dO = O8[sl][f] - O0[sl][f]
        dG = G8[sl][f] - G0[sl][f]
        m = np.abs(dO).max()
        say("  field %d: LES term max %.3e, rhs max %.3e, |dG - dO| %.2e" % (f, m, np.abs(O8[sl][f]).max(),
                                                                           np.abs(dG - dO).max()))
        assert m > 0
        assert np.abs(dG - dO).max() <= 1e-10 * m, (case, f)
    for f in range(I.NU):
        if f not in (28, 29, 30):
            assert np.array_equal(G8[sl][f], G0[sl][f]), f
