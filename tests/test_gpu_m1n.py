"""GPU parity of the neutrino number densities (Sec. 2.3 number current and
source, Sec. 2.2 electron-fraction source, App. C's implicit update) against
the FP64 oracle: the right-hand side of all 47 fields (per field, max |G - O|
/ max |O| <= 1e-10 over the interior points), its split into explicit and
stiff parts, IMEX(4,4,2) steps (the step's own change sets the scale, as for
the other step tests), and the closed-form relaxation of uniform number
densities at rest under Table I's implicit tableau.
"""
import os
import sys
from fractions import Fraction

import numpy as np
import pytest

from paper_2510_13965_amd import inputs as I

pytestmark = pytest.mark.gpu

RTOL = 1e-10
PAR_N = dict(I.PARAMS, evolve_m1=1, evolve_m1n=1, m_b=1.3)


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


def with_n(orc, ip, U, P, EM, seed):
    g = orc.make_grid(ip.n, ip.dx, ng=ip.ng)
    orc.prim2con(g, orc.make_eos(I.EOS_IDEAL2), U, P, EM, 0)
    U44, aux9 = I.m1_fields(ip, U, P, seed)
    return I.m1n_fields(ip, U44, aux9, seed + 1000)


def oracle_full(orc, ip, U, aux):
    g = orc.make_grid(ip.n, ip.dx, ng=ip.ng)
    e = orc.make_eos(I.EOS_IDEAL2)
    Uo = U.copy()
    Po = np.zeros((I.NP,) + ip.shape)
    orc.con2prim(g, e, Uo, Po, None, None)
    out = np.zeros_like(U)
    ms = orc.rhs_full(g, orc.make_par(PAR_N), e, Uo, Po, aux, out)
    return out, ms, Uo, Po


def compare(ip, G, O, tag, nf=I.NU_M1N):
    sl = (slice(None),) + ip.interior()
    bad, errs = [], {}
    for f in range(nf):
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
    say(tag, "worst %.1e" % max(errs.values()), "Ye and N fields",
        {k: "%.1e" % v for k, v in errs.items() if k == 23 or k >= 44})
    assert not bad, (tag, bad)


@pytest.mark.parametrize("case", ["flat", "star"])
def test_m1n_rhs_parity(orc, dev, case):
    import torch
    from paper_2510_13965_amd.step import PatchRun

    if case == "flat":
        say("case m1n rhs, perturbed flat 20^3")
        ip, U, P, EM = I.perturbed_flat_state(n=20, rich=True)
        U47, aux = with_n(orc, ip, U, P, EM, I.SEED0 + 160)
    else:
        say("case m1n rhs, star 36^3")
        ip, U, P, EM = I.tov_star_state(n=36)
        U47, aux = with_n(orc, ip, U, P, EM, I.SEED0 + 161)
    O, mso, _, _ = oracle_full(orc, ip, U47, aux)
    r = PatchRun(ip, U47, I.EOS_IDEAL2, PAR_N, aux=aux)
    r.rhs_eval(r.Un)
    torch.cuda.synchronize()
    compare(ip, r.k.cpu().numpy(), O, case)
    assert float(r.vmax.item()) == pytest.approx(mso, rel=1e-12)


def test_m1n_rhs_split_parity(orc, dev):
    """Explicit part (47 fields) and stiff part (15 fields: the energy
    moments' collision terms, then the number densities' alpha sqrt(gamma) C)."""
    import torch
    from paper_2510_13965_amd import mhd

    say("case m1n rhs split, star 28^3")
    ip, U, P, EM = I.tov_star_state(n=28)
    U47, aux = with_n(orc, ip, U, P, EM, I.SEED0 + 162)
    g = orc.make_grid(ip.n, ip.dx, ng=ip.ng)
    e = orc.make_eos(I.EOS_IDEAL2)
    Uo = U47.copy()
    Po = np.zeros((I.NP,) + ip.shape)
    orc.con2prim(g, e, Uo, Po, None, None)
    Fo = np.zeros_like(U47)
    Ro = np.zeros((15,) + ip.shape)
    orc.rhs_split(g, orc.make_par(PAR_N), e, Uo, Po, aux, Fo, Ro)
    pt = mhd.patch_of(ip)
    Ud = torch.as_tensor(Uo).cuda()
    Pd = torch.as_tensor(Po).cuda()
    F = torch.zeros_like(Ud)
    R = torch.zeros((15,) + ip.shape, dtype=torch.float64, device="cuda")
    mhd.rhs_split(pt, mhd.make_params(PAR_N), mhd.make_eos(I.EOS_IDEAL2), Ud, Pd, torch.as_tensor(aux).cuda(), F, R,
                  None, mhd.workspace_for(pt, m1=True, m1n=True))
    torch.cuda.synchronize()
    compare(ip, F.cpu().numpy(), Fo, "split explicit")
    compare(ip, R.cpu().numpy(), Ro, "split stiff", nf=15)


def compare_step(ip, U0, G, O, tag):
    sl = (slice(None),) + ip.interior()
    worst = 0.0
    for f in range(I.NU_M1N):
        d = np.abs(G[sl][f] - O[sl][f]).max()
        scale = np.abs(O[sl][f] - U0[sl][f]).max()
        bound = 4e-10 * scale + 8 * np.finfo(float).eps * np.abs(O[sl][f]).max()
        if scale > 0:
            worst = max(worst, d / scale)
        assert d <= bound, (tag, f, d, scale)
    say(tag, "worst |G-O| / max|dU| = %.1e" % worst)


@pytest.mark.parametrize("case", ["flat", "star"])
def test_m1n_imex_step_parity(orc, dev, case):
    import torch
    from paper_2510_13965_amd.step import ImexRun

    if case == "flat":
        say("case m1n imex step, perturbed flat 16^3 periodic, opacities x10")
        ip, U, P, EM = I.perturbed_flat_state(n=16, rich=True)
        U47, aux = with_n(orc, ip, U, P, EM, I.SEED0 + 163)
        aux[0::3][:3] *= 10.0
        aux[9:] *= 10.0
        periodic = True
    else:
        say("case m1n imex step, star 28^3 frozen ghosts")
        ip, U, P, EM = I.tov_star_state(n=28)
        U47, aux = with_n(orc, ip, U, P, EM, I.SEED0 + 164)
        periodic = False
    dt = 0.25 * ip.dx[0]
    g = orc.make_grid(ip.n, ip.dx, ng=ip.ng)
    e = orc.make_eos(I.EOS_IDEAL2)
    Uo = U47.copy()
    nf_o = orc.imex_step(g, orc.make_par(PAR_N), e, Uo, aux, dt, periodic=periodic)
    r = ImexRun(ip, U47, aux, I.EOS_IDEAL2, PAR_N, periodic=periodic)
    r.step(dt)
    torch.cuda.synchronize()
    assert nf_o == 0 and int(r.nfail.item()) == 0
    compare_step(ip, U47, r.Un.cpu().numpy(), Uo, case)


def test_m1n_uniform_relaxation_closed_form(dev):
    """Uniform fluid and isotropic radiation at rest, lapse 0.9, no energy
    opacities, number opacity kappa0 and emissivity eta0: one GPU IMEX step
    multiplies the distance to eta0/kappa0 by R(z), z = -alpha kappa0 dt, of
    Table I's implicit tableau (at kappa0 dt = 0.3, 10 and 1e4), and leaves E,
    F_i as they are."""
    import torch
    from paper_2510_13965_amd import mhd
    from paper_2510_13965_amd.step import ImexRun

    say("case m1n uniform relaxation")
    path = os.path.join(os.path.dirname(__file__), "golden", "table1_imex442.txt")
    lines = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    i0 = [k for k, l in enumerate(lines) if l[0] == "implicit_A"][0]
    A = np.array([[float(Fraction(x)) for x in lines[i0 + 1 + r]] for r in range(4)])
    b = np.array([float(Fraction(x)) for x in [l for l in lines if l[0] == "implicit_b"][0][1:]])
    ip = I.Patch((6, 6, 6), (0.1,) * 3, (0.0,) * 3)
    U = np.zeros((I.NU_M1N,) + ip.shape)
    P = np.zeros((I.NP,) + ip.shape)
    EM = np.zeros((I.NEM,) + ip.shape)
    I.flat_spacetime(U)
    alpha = 0.9
    U[I.ALPHA] = alpha
    P[I.RHO], P[I.EPS], P[I.YE] = 1e-3, 0.1, 0.1
    Ud = torch.as_tensor(U).cuda()
    mhd.prim2con(mhd.patch_of(ip), mhd.make_eos(I.EOS_IDEAL2), Ud, torch.as_tensor(P).cuda(),
                 torch.as_tensor(EM).cuda(), 0)
    U = Ud.cpu().numpy()
    N0, eta0, dt = 2e-6, 1e-7, 0.025
    for kdt in (0.3, 10.0, 1e4):
        aux = np.zeros((I.NAUX_N,) + ip.shape)
        for s in range(3):
            U[32 + 4 * s] = 2e-5
            U[33 + 4 * s:36 + 4 * s] = 0.0
            U[44 + s] = N0 * (s + 1)
            aux[9 + 2 * s] = kdt / dt * (s + 1)
            aux[10 + 2 * s] = eta0
        r = ImexRun(ip, U, aux, I.EOS_IDEAL2, dict(PAR_N, couple_matter=0), periodic=True)
        r.step(dt)
        torch.cuda.synchronize()
        out = r.Un.cpu().numpy()
        sl = ip.interior()
        for s in range(3):
            k = kdt / dt * (s + 1)
            z = -alpha * k * dt
            R = 1.0 + z * b @ np.linalg.solve(np.eye(4) - z * A, np.ones(4))
            want = eta0 / k + R * (N0 * (s + 1) - eta0 / k)
            got = out[44 + s][sl]
            tol = 64 * np.finfo(float).eps * (1.0 + abs(z)) * N0 * (s + 1)
            assert np.abs(got - want).max() <= tol, (kdt, s, got.ravel()[0], want)
            assert np.array_equal(out[32 + 4 * s][sl], U[32 + 4 * s][sl])


# ---------------------------------------------------------------- batched levels

@pytest.fixture(scope="module")
def level_n_states(dev, orc):
    """Five uneven boxes of the star (edges 16..48) with three grey species and
    their number densities; cons built by the oracle."""
    boxes = I.amr_level_boxes(seed=I.SEED0 + 37, nboxes=5, edges=(16, 24, 32, 48))
    Ab = I.star_field_amplitude()
    out = []
    for b, box in enumerate(boxes):
        ip, U, P, EM = I.amr_box_state(box, Ab)
        U47, aux = with_n(orc, ip, U, P, EM, I.SEED0 + 370 + b)
        out.append((ip, U47, aux))
    say("level N boxes", [ip.n for ip, _, _ in out])
    return out


def n_level_run(states, **kw):
    from paper_2510_13965_amd.step import LevelRun

    return LevelRun([s[0] for s in states], [s[1] for s in states], I.EOS_IDEAL2, PAR_N,
                    auxs=[s[2] for s in states], **kw)


def test_m1n_level_rhs_bitwise_and_oracle(orc, level_n_states):
    """The batched level's right-hand side with the number densities equals
    per-box mhd_rhs bit for bit (47 fields, primitives, flags, speed), and its
    smallest box matches the oracle to 1e-10 per field."""
    import torch
    from paper_2510_13965_amd.step import PatchRun

    say("case level N rhs vs per-box and oracle, 5 boxes")
    ref, vref = [], 0.0
    for ip, U, aux in level_n_states:
        r = PatchRun(ip, U, I.EOS_IDEAL2, PAR_N, aux=aux)
        r.rhs_eval(r.Un)
        torch.cuda.synchronize()
        vref = max(vref, float(r.vmax.item()))
        ref.append((r.k.cpu().numpy(), r.P.cpu().numpy(), r.flags.cpu().numpy()))
    run = n_level_run(level_n_states)
    ms = torch.zeros(1, dtype=torch.float64, device="cuda")
    run.level.rhs(0, ms)
    torch.cuda.synchronize()
    for b, box in enumerate(run.boxes):
        assert np.array_equal(ref[b][0], box["k"].cpu().numpy()), b
        assert np.array_equal(ref[b][1], box["P"].cpu().numpy()), b
        assert np.array_equal(ref[b][2], box["flags"].cpu().numpy()), b
    assert float(ms.item()) == vref
    small = min(range(len(level_n_states)), key=lambda b: level_n_states[b][0].npts)
    ip, U, aux = level_n_states[small]
    O, _, _, _ = oracle_full(orc, ip, U, aux)
    compare(ip, run.boxes[small]["k"].cpu().numpy(), O, "level box %s" % (ip.n,))


def test_m1n_level_rk4_and_imex_bitwise(level_n_states):
    """Two RK4 steps and two IMEX(4,4,2) steps (opacities x100) of the level,
    eager and as replayed graphs, against per-box steps: bitwise."""
    import torch
    from paper_2510_13965_amd.step import ImexRun, PatchRun

    say("case level N rk4 + imex vs per-box, 5 boxes")
    dt = 0.25 * 0.25
    boxes = [PatchRun(ip, U, I.EOS_IDEAL2, PAR_N, aux=aux) for ip, U, aux in level_n_states]
    eager = n_level_run(level_n_states)
    graph = n_level_run(level_n_states)
    stream = torch.cuda.Stream()
    for step in range(2):
        for r in boxes:
            r.step(dt)
        eager.level.rk4_step(dt, None)
        stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(stream):
            graph.level.rk4_step(dt, None, use_graph=True, stream=stream)
        stream.synchronize()
        torch.cuda.synchronize()
        for b, r in enumerate(boxes):
            ref = r.Un.cpu().numpy()
            assert np.isfinite(ref).all()
            assert np.array_equal(ref, eager.boxes[b]["U"].cpu().numpy()), ("rk4 eager", step, b)
            assert np.array_equal(ref, graph.boxes[b]["U"].cpu().numpy()), ("rk4 graph", step, b)
    states = [(ip, U, aux * 1e2) for ip, U, aux in level_n_states]
    par = dict(PAR_N)
    ibox = [ImexRun(ip, U, aux, I.EOS_IDEAL2, par) for ip, U, aux in states]
    ie = n_level_run(states, imex=True)
    ig = n_level_run(states, imex=True)
    nf_e = torch.zeros(1, dtype=torch.int64, device="cuda")
    nf_g = torch.zeros(1, dtype=torch.int64, device="cuda")
    for step in range(2):
        for r in ibox:
            r.step(dt)
        ie.level.imex_step(dt, None, nf_e)
        stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(stream):
            ig.level.imex_step(dt, None, nf_g, use_graph=True, stream=stream)
        stream.synchronize()
        torch.cuda.synchronize()
        for b, r in enumerate(ibox):
            ref = r.Un.cpu().numpy()
            assert np.isfinite(ref).all()
            assert np.array_equal(ref, ie.boxes[b]["U"].cpu().numpy()), ("imex eager", step, b)
            assert np.array_equal(ref, ig.boxes[b]["U"].cpu().numpy()), ("imex graph", step, b)
        assert int(nf_e.item()) == int(nf_g.item()) == sum(int(r.nfail.item()) for r in ibox)


# ---------------------------------------------------------------- coupled exchange

@pytest.mark.parametrize("case", ["star", "star+N"])
def test_coupled_exchange_imex_step_parity(orc, dev, case):
    """IMEX(4,4,2) with the fluid's share of the exchange implicit too
    (MHD_COUPLE_EXCHANGE): the 28^3 star at opacities x100, with and without
    the number densities, against the oracle's step; the split right-hand
    side's stiff fluid slots against the oracle's."""
    import torch
    from paper_2510_13965_amd import mhd
    from paper_2510_13965_amd.step import ImexRun

    nd = case.endswith("N")
    say("case coupled exchange imex step,", case, "28^3, opacities x100")
    ip, U, P, EM = I.tov_star_state(n=28)
    if nd:
        U0, aux = with_n(orc, ip, U, P, EM, I.SEED0 + 171)
        par = dict(PAR_N, couple_exchange=1)
    else:
        g = orc.make_grid(ip.n, ip.dx, ng=ip.ng)
        orc.prim2con(g, orc.make_eos(I.EOS_IDEAL2), U, P, EM, 0)
        U0, aux = I.m1_fields(ip, U, P, I.SEED0 + 171)
        par = dict(I.PARAMS, evolve_m1=1, couple_exchange=1)
    aux = aux * 100.0
    nf = U0.shape[0]
    dt = 0.25 * ip.dx[0]
    g = orc.make_grid(ip.n, ip.dx, ng=ip.ng)
    e = orc.make_eos(I.EOS_IDEAL2)
    # split right-hand side at the initial state
    op = orc.make_par(par)
    nr = orc.imex_stiff_fields(op)
    assert nr == mhd.imex_stiff_fields(nf, True) == (20 if nd else 16)
    Uo = U0.copy()
    Po = np.zeros((I.NP,) + ip.shape)
    orc.con2prim(g, e, Uo, Po, None, None)
    Fo, Ro = np.zeros_like(U0), np.zeros((nr,) + ip.shape)
    orc.rhs_split(g, op, e, Uo, Po, aux, Fo, Ro)
    pt = mhd.patch_of(ip)
    F = torch.zeros((nf,) + ip.shape, dtype=torch.float64, device="cuda")
    R = torch.zeros((nr,) + ip.shape, dtype=torch.float64, device="cuda")
    mhd.rhs_split(pt, mhd.make_params(par), mhd.make_eos(I.EOS_IDEAL2), torch.as_tensor(Uo).cuda(),
                  torch.as_tensor(Po).cuda(), torch.as_tensor(aux).cuda(), F, R, None,
                  mhd.workspace_for(pt, m1=True, m1n=nd))
    torch.cuda.synchronize()
    compare(ip, F.cpu().numpy(), Fo, "split explicit", nf=nf)
    compare(ip, R.cpu().numpy(), Ro, "split stiff", nf=nr)
    # one step
    Uo = U0.copy()
    nf_o = orc.imex_step(g, op, e, Uo, aux, dt)
    r = ImexRun(ip, U0, aux, I.EOS_IDEAL2, par)
    r.step(dt)
    torch.cuda.synchronize()
    assert nf_o == 0 and int(r.nfail.item()) == 0
    compare_step_n(ip, U0, r.Un.cpu().numpy(), Uo, case, nf)


def compare_step_n(ip, U0, G, O, tag, nf):
    sl = (slice(None),) + ip.interior()
    worst = 0.0
    for f in range(nf):
        d = np.abs(G[sl][f] - O[sl][f]).max()
        scale = np.abs(O[sl][f] - U0[sl][f]).max()
        bound = 4e-10 * scale + 8 * np.finfo(float).eps * np.abs(O[sl][f]).max()
        if scale > 0:
            worst = max(worst, d / scale)
        assert d <= bound, (tag, f, d, scale)
    say(tag, "worst |G-O| / max|dU| = %.1e" % worst)


def test_coupled_exchange_conserves_on_gpu(dev):
    """Uniform fluid and radiation at rest on a flat periodic patch, no
    gravity response, kappa_a dt = 10, 20, 30 and an equilibrium below the
    radiation: one GPU IMEX step with the coupled exchange relaxes Ebar by
    R(z) of Table I's implicit tableau and conserves taubar + sum Ebar to
    rounding, while the fluid takes most of the radiation's energy."""
    import torch
    from paper_2510_13965_amd import mhd
    from paper_2510_13965_amd.step import ImexRun

    say("case coupled exchange, uniform relaxation on the GPU")
    ip = I.Patch((8, 8, 8), (0.1,) * 3, (0.0,) * 3)
    U = np.zeros((44,) + ip.shape)
    P = np.zeros((I.NP,) + ip.shape)
    I.flat_spacetime(U)
    P[I.RHO] = 1e-3
    P[I.EPS] = 0.1
    P[I.WLOR] = 1.0
    P[I.YE] = 0.1
    pt = mhd.patch_of(ip)
    Ud = torch.as_tensor(U).cuda()
    mhd.prim2con(pt, mhd.make_eos(I.EOS_IDEAL2), Ud, torch.as_tensor(P).cuda(),
                 torch.zeros((4,) + ip.shape, dtype=torch.float64, device="cuda"), 0)
    U = Ud.cpu().numpy()
    aux = np.zeros((9,) + ip.shape)
    dt = 0.025
    E0 = [1e-5, 2e-5, 3e-5]
    for s in range(3):
        U[32 + 4 * s] = E0[s]
        aux[3 * s] = 10.0 * (s + 1) / dt
        aux[3 * s + 2] = 1e-7 * aux[3 * s]
    r = ImexRun(ip, U, aux, I.EOS_IDEAL2, dict(I.PARAMS, couple_matter=0, couple_exchange=1), periodic=True)
    r.step(dt)
    torch.cuda.synchronize()
    X = r.Un.cpu().numpy()[(slice(None),) + ip.interior()]
    a = U[(slice(None),) + ip.interior()]
    from oracle import orc

    _, A, _, b = orc.imex_tableau(0)
    for s in range(3):
        z = -10.0 * (s + 1)
        Rz = 1.0 + z * b @ np.linalg.solve(np.eye(len(b)) - z * A, np.ones(len(b)))
        want = 1e-7 + Rz * (E0[s] - 1e-7)
        tol = 64 * np.finfo(float).eps * (1.0 + abs(z)) * E0[s]
        assert np.abs(X[32 + 4 * s] - want).max() <= tol
    tot = lambda x: x[24] + sum(x[32 + 4 * s] for s in range(3))
    scale = np.abs(a[24]).max() + sum(E0)
    assert np.abs(X[24] - a[24]).max() > 0.5 * sum(E0)
    assert np.abs(tot(X) - tot(a)).max() <= 64 * np.finfo(float).eps * 31.0 * scale
