"""GPU parity of the grey M1 part (three species) against the FP64 oracle.

Bar as for the rest of the RHS: per field, max |G - O| / max |O| <= 1e-10 over
the interior points, for all 44 fields (the radiation also feeds the CCZ4
matter terms and exchanges energy and momentum with the fluid).
"""
import sys

import numpy as np
import pytest

from paper_2510_13965_amd import inputs as I

pytestmark = pytest.mark.gpu

RTOL = 1e-10
PAR_M1 = dict(I.PARAMS, evolve_m1=1)


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


def with_m1(orc, ip, U, P, EM, seed, eos_cfg=I.EOS_IDEAL2):
    g = orc.make_grid(ip.n, ip.dx, ng=ip.ng)
    orc.prim2con(g, orc.make_eos(eos_cfg), U, P, EM, 0)
    return I.m1_fields(ip, U, P, seed)


def oracle_full(orc, ip, U, aux, par_cfg=PAR_M1, eos_cfg=I.EOS_IDEAL2):
    g = orc.make_grid(ip.n, ip.dx, ng=ip.ng)
    e = orc.make_eos(eos_cfg)
    Uo = U.copy()
    Po = np.zeros((I.NP,) + ip.shape)
    orc.con2prim(g, e, Uo, Po, None, None)
    out = np.zeros_like(U)
    ms = orc.rhs_full(g, orc.make_par(par_cfg), e, Uo, Po, aux, out)
    return out, ms


def gpu_full(ip, U, aux, par_cfg=PAR_M1, eos_cfg=I.EOS_IDEAL2):
    import torch
    from paper_2510_13965_amd import mhd
    from paper_2510_13965_amd.step import PatchRun

    r = PatchRun(ip, U, eos_cfg, par_cfg, aux=aux)
    r.rhs_eval(r.Un)
    torch.cuda.synchronize()
    return r.k.cpu().numpy(), float(r.vmax.item())


def compare(ip, G, O, tag):
    sl = (slice(None),) + ip.interior()
    bad, errs = [], {}
    for f in range(I.NU_M1):
        g, o = G[sl][f], O[sl][f]
        m = np.abs(o).max()
        if m == 0.0:
            if np.abs(g).max() > 1e-300:
                bad.append((f, "zero field", float(np.abs(g).max())))
            continue
        err = float(np.abs(g - o).max() / m)
        errs[f] = err
        if not err <= RTOL:
            bad.append((f, err))
    say(tag, "worst", "%.1e" % max(errs.values()), "M1 fields",
        {k: "%.1e" % v for k, v in errs.items() if k >= 32})
    assert not bad, (tag, bad)


def test_m1_rhs_parity_perturbed_flat(orc, dev):
    say("case m1 rhs, perturbed flat 24^3")
    ip, U, P, EM = I.perturbed_flat_state(n=24, rich=True)
    U44, aux = with_m1(orc, ip, U, P, EM, seed=I.SEED0 + 60)
    O, mso = oracle_full(orc, ip, U44, aux)
    G, msg = gpu_full(ip, U44, aux)
    compare(ip, G, O, "flat+m1")
    assert msg == pytest.approx(mso, rel=1e-12)


def test_m1_rhs_parity_star(orc, dev):
    say("case m1 rhs, star 40^3")
    ip, U, P, EM = I.tov_star_state(n=40)
    U44, aux = with_m1(orc, ip, U, P, EM, seed=I.SEED0 + 61)
    O, mso = oracle_full(orc, ip, U44, aux)
    G, msg = gpu_full(ip, U44, aux)
    compare(ip, G, O, "star+m1")
    assert msg == pytest.approx(mso, rel=1e-12)


def test_m1_rhs_parity_star_64(orc, dev):
    """The star at the benchmark's patch size (64^3 interior, three species),
    every interior point of all 44 fields against the oracle."""
    say("case m1 rhs, star 64^3")
    ip, U, P, EM = I.tov_star_state(n=64)
    U44, aux = with_m1(orc, ip, U, P, EM, seed=I.SEED0 + 63)
    O, mso = oracle_full(orc, ip, U44, aux)
    G, msg = gpu_full(ip, U44, aux)
    compare(ip, G, O, "star64+m1")
    assert msg == pytest.approx(mso, rel=1e-12)


def test_m1_rk4_step_parity(orc, dev):
    """One RK4 step with 44 fields, frozen ghosts, against the oracle's step."""
    import torch
    from paper_2510_13965_amd.step import PatchRun

    say("case m1 rk4 step, perturbed flat 20^3")
    ip, U, P, EM = I.perturbed_flat_state(n=20, rich=True)
    U44, aux = with_m1(orc, ip, U, P, EM, seed=I.SEED0 + 62)
    dt = 0.25 * ip.dx[0]
    g = orc.make_grid(ip.n, ip.dx, ng=ip.ng)
    e = orc.make_eos(I.EOS_IDEAL2)
    par = orc.make_par(PAR_M1)
    Un = U44.copy()
    Us = U44.copy()
    acc = np.zeros_like(U44)
    k = np.zeros_like(U44)
    Po = np.zeros((I.NP,) + ip.shape)
    for s in range(4):
        X = Un if s == 0 else Us
        orc.con2prim(g, e, X, Po, None, None)
        orc.rhs_full(g, par, e, X, Po, aux, k)
        orc.rk4_stage_interior(g, I.NU_M1, s, dt, Un, k, acc, Us if s < 3 else Un)
    r = PatchRun(ip, U44, I.EOS_IDEAL2, PAR_M1, aux=aux)
    r.step(dt)
    torch.cuda.synchronize()
    G = r.Un.cpu().numpy()
    sl = (slice(None),) + ip.interior()
    for f in range(I.NU_M1):
        d = np.abs(G[sl][f] - Un[sl][f]).max()
        scale = np.abs(Un[sl][f] - U44[sl][f]).max()
        assert d <= 4e-10 * scale + 8 * np.finfo(float).eps * np.abs(Un[sl][f]).max(), (f, d, scale)
